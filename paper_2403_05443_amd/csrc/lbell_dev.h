// lbell_dev.h - device-side data structures and lattice constants of the HIP
// library (internal; not part of the C ABI).  Written for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbd {

constexpr int NQMAX = 27;        // velocities of the largest set (D3Q27)
constexpr int TILE = 256;        // sites per K1 work-group
constexpr int PBLOCK = 512;      // threads per particle work-group
constexpr int PWAVES = PBLOCK / 64;
constexpr int KREG = 2;          // links per thread held in registers across phases
constexpr int KOVF = 4;          // links past those whose loads one thread issues together
constexpr double BAND_M = 1.0;   // narrow band of the remap scan: nodes within this margin (lattice units)
constexpr int KSCAN = 4;         // window sites per thread whose node-map loads the solid scan issues together
constexpr int STAGE = 4096;      // link codes staged in LDS per copy-out round
constexpr int SITE_BITS = 27;    // link code: site | dir << 27
constexpr uint32_t SITE_MASK = (1u << SITE_BITS) - 1u;

// Velocity sets, order fixed by the ABI (link codes carry it): rest, 6 axis,
// 12 edge vectors (D3Q19, Q = 19); D3Q27 (Q = 27) appends the 8 corners
// (1,1,1), (1,1,-1), (1,-1,1), (-1,1,1), each followed by its opposite.  The
// opposite of odd i is i + 1, so one table serves both sets.
__host__ __device__ constexpr int corner(int i, int flip) {  // component of corner i >= 19
    return ((i & 1) ? 1 : -1) * (((i - 19) >> 1) == flip ? -1 : 1);
}
__host__ __device__ constexpr int cx_def(int i) {
    return i >= 19 ? corner(i, 3)
         : (i == 1 || i == 7 || i == 9 || i == 11 || i == 13 ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14 ? -1 : 0));
}
__host__ __device__ constexpr int cy_def(int i) {
    return i >= 19 ? corner(i, 2)
         : (i == 3 || i == 7 || i == 10 || i == 15 || i == 17 ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18 ? -1 : 0));
}
__host__ __device__ constexpr int cz_def(int i) {
    return i >= 19 ? corner(i, 1)
         : (i == 5 || i == 11 || i == 14 || i == 15 || i == 18 ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17 ? -1 : 0));
}
// The same components packed two bits per direction (c + 1), so that a
// direction known only at run time costs a shift and a mask rather than a
// chain of compares (which diverges across a wave's lanes).
template <int AXIS>
__host__ __device__ constexpr unsigned long long pack_c() {
    unsigned long long v = 0;
    for (int i = 0; i < 27; ++i)
        v |= (unsigned long long)((AXIS == 0 ? cx_def(i) : (AXIS == 1 ? cy_def(i) : cz_def(i))) + 1) << (2 * i);
    return v;
}
constexpr unsigned long long CX_PACK = pack_c<0>(), CY_PACK = pack_c<1>(), CZ_PACK = pack_c<2>();
__host__ __device__ constexpr int cx(int i) { return (int)((CX_PACK >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cy(int i) { return (int)((CY_PACK >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cz(int i) { return (int)((CZ_PACK >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216
template <int Q>
__host__ __device__ constexpr double wgt(int i) {
    return Q == 27 ? (i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0)))
                   : (i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0));
}
// W w_i as an exact integer: W = 36 for D3Q19 (12, 2, 1), 216 for D3Q27 (64, 16, 4, 1)
template <int Q>
constexpr int WSCALE = Q == 27 ? 216 : 36;
template <int Q>
__host__ __device__ constexpr int wint(int i) {
    return Q == 27 ? (i == 0 ? 64 : (i <= 6 ? 16 : (i <= 18 ? 4 : 1))) : (i == 0 ? 12 : (i <= 6 ? 2 : 1));
}

enum Flags : int {
    F_OVERLAP = 1,      // a node claimed by two particles or a particle and a wall
    F_NONFINITE = 2,    // singular 6x6 or non-finite / too fast particle
    F_LINKS = 4,        // link capacity exceeded
    F_WINDOW = 8,       // remap window larger than the LDS budget
};

struct BoxDesc {
    int nx, ny, nz, n;
    long long foff;       // element offset of the box's population block
    long long stride;     // elements between direction planes
    long long ooff;       // element offset of the box's node map
    int walls, n_wall;
    int tile0, ntiles;
    int counterforce, pad0;
    double wall_lo[3], wall_hi[3];
    double fext[3];       // sum of external forces on this machine's particles
    double gcf[3];        // counter-force density -fext / (n - n_wall), or 0
    uint32_t mnx, mny;    // site -> (x, y, z) by multiplication: see magic_div
    int lnx, lny;
    long long coff;       // offset of the box's cells (8^3 nodes each) in the owner-change stamps
    int cnx, cny;         // cells along x and y
};

// Division of 0 <= n < 2^27 (a site index, SITE_BITS) by d >= 1 as one
// multiply and shift: m = ceil(2^L / d) with L = 27 + ceil(log2 d) (m < 2^29).
// Exact: n / d differs from n m / 2^L by n (m d - 2^L) / (d 2^L), and
// n (m d - 2^L) < 2^27 d <= 2^L keeps it below the gap to the next integer.
inline void magic_div(int d, uint32_t& m, int& L) {
    int c = 0;
    while ((1ll << c) < d) ++c;
    L = SITE_BITS + c;
    m = (uint32_t)(((1ull << L) + (unsigned long long)d - 1) / (unsigned long long)d);
}
__device__ __forceinline__ int div_magic(int n, int d, uint32_t m, int L, int& r) {
    const int q = (int)(((unsigned long long)(uint32_t)n * m) >> L);
    r = n - q * d;
    return q;
}

struct BoxRT {            // mutated by kernels
    int n_solid;
    int pad[3];
};

struct PartDev {
    double xc[3];         // centre, wrapped into the box
    double xu[3];         // centre, unwrapped
    double q[4];          // orientation (scalar first, body -> lab)
    double qprev[4];      // orientation one step earlier (q on the first step)
    double U[3], W[3];    // velocity, angular velocity (lab)
    double axes[3];       // semi-axes a, b, c along body x, y, z
    double ia2[3];        // 1 / axis^2, computed on the host
    double M, Ib[3];      // mass and body inertia
    double Fext[3], Text[3];
    double B1, B2;        // squirmer modes
    // moments of the current link set about the unwrapped centre xref at
    // which it was enumerated (rho = link midpoint - xref, weights W w):
    // zm1 = sum c (rho x c)^T (3x3), zm2 = sum (rho x c)(rho x c)^T (upper
    // triangle); with zm0 = sum c c^T they give the [F;T] x [U;W] drag
    // matrix zeta at any later centre
    double zm1[9], zm2[6], xref[3];
    // pose at the last test of the window (unwrapped centre, orientation),
    // the smallest distance-like margin of its nodes to the surface and the
    // largest distance of its nodes from the centre (remap skip test)
    double sref[3], qref[4], smargin, srho;
    // narrow band of the last full test: the pose it was taken at, its
    // window (origin, edges) and the largest distance of that window's nodes
    // from the centre; the band itself (window nodes whose margin was below
    // BAND_M) is a bitmask over that window in the band area
    double bref[3], bqref[4], bsrho;
    int blo[3], bwn[3], bvalid, bpad;
    double dm, Pp[3], Lp[3];  // pending mass / momentum / angular momentum of transitions
    double F[3], T[3];    // hydrodynamic force and torque of the last step
    double wsum;          // sum of w_b over the current links
    int box, nlinks, lcap, n_solid;
    int zm0[6];           // sum 36 w c c^T (upper triangle), exact
    // set by the remap scan of the step in boxes with several particles:
    // some node changed side / some node is a claim candidate
    int nchg, ncand;
    long long lbase;      // offset of this particle's links in the pool
};

// Fallback monitor of a warm-started box (one record per box).
enum MonStatus : int {
    MON_OFF = 0,          // no warm start to watch
    MON_PENDING = 1,      // warm-started, not decided yet
    MON_ACCEPTED = 2,     // within tol of the prediction at the decision
    MON_FALLBACK = 3,     // missed while the run was still evolving: reset to the plain start
    MON_STEADY_MISS = 4,  // missed, but the run was already steady: kept, its sample queued for training
};
struct BoxMon {
    double E_ref;          // flow energy sum |j|^2 at the reference check
    double tol;            // relative tolerance of the prediction and of the residuals
    double res_flow;       // residuals of the decision: relative changes since the reference
    double res_part;
    long long t0;          // step of the warm start
    long long t_ref;       // step of the reference check (-1: not yet)
    long long t_decided;   // step of the decision (-1 before it)
    int W0;                // steps from the warm start before the decision
    int Wref;              // steps from the warm start before the reference check
    int status;            // MonStatus
    int reset;             // set by the last check when it fell back
};

struct KParams {
    double omega, omega_m;    // 1/tau (TRT: 1/tau+), TRT 1/tau-
    double scale, inv_scale;  // half formats: stored = scale * deviation
    double rho0;
    int collision, storage;
    int conv;                 // storage convention of the current populations (CV_*)
    int q;                    // velocity set: 19 or 27
    int rot;                  // inertia term of the rotational update (LB_ROT_*)
};

// Storage conventions of the population array.  The post-collision
// population f*_i(x) of node x is held in slot (direction plane, site)
//   CV_PULL  (i, x)          two buffers; a step pulls from x - c_i of one and
//                            writes the other
//   CV_EVEN  (opp(i), x)     one buffer, after an in-place even step
//   CV_ODD   (i, x + c_i)    one buffer, after an in-place odd step
// An in-place even step reads each node's own slots and writes them back
// (CV_ODD -> CV_EVEN); an odd step gathers from and scatters to the
// neighbours (CV_EVEN -> CV_ODD).  Either way every slot is read and written
// by one node only.  The pre-collision f_i(x) a node reads at the next step
// is f*_i(x - c_i): slot (i, x - c_i), (opp(i), x - c_i) or (i, x).
constexpr int CV_PULL = 0, CV_EVEN = 1, CV_ODD = 2;

__host__ __device__ inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Slot of f*_i at node (x, y, z) of an nx x ny x nz box.
__host__ __device__ inline void post_slot(int cv, int i, int x, int y, int z, int nx, int ny, int nz, int& dir,
                                          int& site) {
    if (cv == CV_ODD) {
        dir = i;
        site = wrap(x + cx(i), nx) + nx * (wrap(y + cy(i), ny) + ny * wrap(z + cz(i), nz));
    } else {
        dir = cv == CV_EVEN ? opp(i) : i;
        site = x + nx * (y + ny * z);
    }
}

// Slot of the pre-collision f_i of node (x, y, z) (no wall in between).
__host__ __device__ inline void pre_slot_open(int cv, int i, int x, int y, int z, int nx, int ny, int nz, int& dir,
                                              int& site) {
    if (cv == CV_ODD) {
        dir = i;
        site = x + nx * (y + ny * z);
    } else {
        dir = cv == CV_EVEN ? opp(i) : i;
        site = wrap(x - cx(i), nx) + nx * (wrap(y - cy(i), ny) + ny * wrap(z - cz(i), nz));
    }
}

// Rounding dither of the half formats: one murmur3 32-bit finalisation per
// (site of its box, step) seeds the site; the direction pair (2k-1, 2k) shares
// p = (seed + k * golden) * an odd constant: the first takes its high 16
// bits, the second its low 16 bits (uniform too: the low half of the product
// is a bijection of the seed's uniform low half) moved up, the conversions
// drawing on the high bits.  A function of (site, direction, step) only, so
// every collide-stream variant rounds identically.
__device__ __forceinline__ uint32_t dither_seed(uint32_t site, uint32_t step) {
    uint32_t h = site * 0x9E3779B1u + step * 0x85EBCA77u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}
// the dither word of direction dir (random in its high 16 bits); dir is a
// compile-time constant in the kernels, so a pair's product is formed once
__device__ __forceinline__ uint32_t dither_bits(uint32_t seed, int dir) {
    const uint32_t p = (seed + (uint32_t)((dir + 1) >> 1) * 0x9E3779B9u) * 0x2C1B3C6Du;
    return (dir & 1) ? p : (p << 16);
}

}  // namespace lbd

namespace lbd {

// Population storage formats (values of lb_config.storage).
constexpr int ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3;

// Stored value <-> deviation f_i - w_i rho0 in the collision precision R.
template <int ST> struct Store;
template <> struct Store<ST_F64> {
    using T = double;
    using R = double;
    static __device__ __forceinline__ R ld(const T* p, R) { return *p; }
    static __device__ __forceinline__ void st(T* p, R v, R) { *p = v; }
    static __device__ __forceinline__ void st_dither(T* p, R v, R, uint32_t) { *p = v; }
    static __device__ __forceinline__ double ld64(const T* p, double) { return *p; }
    static __device__ __forceinline__ double cv64(T v, double) { return v; }
    static __device__ __forceinline__ void st64(T* p, double v, double) { *p = v; }
};
template <> struct Store<ST_F32> {
    using T = float;
    using R = float;
    static __device__ __forceinline__ R ld(const T* p, R) { return *p; }
    static __device__ __forceinline__ void st(T* p, R v, R) { *p = v; }
    static __device__ __forceinline__ void st_dither(T* p, R v, R, uint32_t) { *p = v; }
    static __device__ __forceinline__ double ld64(const T* p, double) { return (double)*p; }
    static __device__ __forceinline__ double cv64(T v, double) { return (double)v; }
    static __device__ __forceinline__ void st64(T* p, double v, double) { *p = (float)v; }
};
template <> struct Store<ST_F16> {
    using T = _Float16;
    using R = float;
    static __device__ __forceinline__ R ld(const T* p, R inv) { return (float)*p * inv; }
    static __device__ __forceinline__ void st(T* p, R v, R s) { *p = (_Float16)(v * s); }
    // Stochastic rounding: a value rounds up with probability equal to its
    // distance from the lower FP16 neighbour (over one ulp), so increments far
    // below one FP16 ulp (the counter-force) survive in expectation instead
    // of being rounded away in a steady flow.  The conversion instruction
    // does it in one step, normal and subnormal range alike, drawing on the
    // high bits of r (checked: unbiased to the sampling noise over 2^20 draws,
    // and the low 16 bits of r alone have no effect); a value rounded up past
    // the largest finite half becomes infinite, which the non-finite watchdog
    // reports.
    static __device__ __forceinline__ void st_dither(T* p, R v, R s, uint32_t r) {
        typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
        half2_t o = {(_Float16)0.0f, (_Float16)0.0f};
        o = __builtin_amdgcn_cvt_sr_f16_f32(o, v * s, r, false);
        *p = o[0];
    }
    static __device__ __forceinline__ double ld64(const T* p, double inv) { return (double)(float)*p * inv; }
    static __device__ __forceinline__ double cv64(T v, double inv) { return (double)(float)v * inv; }
    static __device__ __forceinline__ void st64(T* p, double v, double s) { *p = (_Float16)(float)(v * s); }
};
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return (uint16_t)(u >> 16);
}
template <> struct Store<ST_BF16> {
    using T = uint16_t;
    using R = float;
    static __device__ __forceinline__ R ld(const T* p, R inv) { return bf16_to_f32(*p) * inv; }
    static __device__ __forceinline__ void st(T* p, R v, R s) { *p = f32_to_bf16(v * s); }
    // stochastic rounding: r's high 16 bits added below the kept mantissa,
    // then cut
    static __device__ __forceinline__ void st_dither(T* p, R v, R s, uint32_t r) {
        const float x = v * s;
        *p = isfinite(x) ? (uint16_t)((__float_as_uint(x) + (r >> 16)) >> 16) : f32_to_bf16(x);
    }
    static __device__ __forceinline__ double ld64(const T* p, double inv) { return (double)bf16_to_f32(*p) * inv; }
    static __device__ __forceinline__ double cv64(T v, double inv) { return (double)bf16_to_f32(v) * inv; }
    static __device__ __forceinline__ void st64(T* p, double v, double s) { *p = f32_to_bf16((float)(v * s)); }
};

__host__ __device__ inline int storage_bytes(int st) { return st == ST_F64 ? 8 : (st == ST_F32 ? 4 : 2); }

}  // namespace lbd
