// k_particle.hip - the particle phase of one time step, one work-group per
// particle (Appendix A, steps 3-9):
//
//   k_particle_solve  F0, T0 over the boundary links (eqs. F0, T0; FP64,
//                     wave shuffles + LDS), lab inertia and its rate
//                     (eqs. Irot, Irotdiff), implicit 6x6 solve (eqs.
//                     Fdiscrete, Tdiscrete), link bounce-back with the
//                     moving-boundary term (eqs. fb, ub, ubsquirmer), then
//                     position and quaternion update (eqs. posupdate,
//                     qnplus0, qnplus1).
//   k_particle_remap  FP64 inside test of eq. ellipsoidsurface over the
//                     particle's window, covered/uncovered node book-keeping,
//                     boundary-link list by LDS-staged compaction in a fixed
//                     (window, direction) order, and the drag matrices of
//                     eqs. drag1-drag4.
//
// Links are packed as site | dir << 27.  All particle quantities are FP64.
#include "lbell_dev.h"
#include "lbell_launch.h"

namespace lbd {

__device__ __forceinline__ int rcx(int b) { return cx(b); }
__device__ __forceinline__ int rcy(int b) { return cy(b); }
__device__ __forceinline__ int rcz(int b) { return cz(b); }
// the weight of direction b in exact integer form (W w_b, W = WSCALE<Q>), and
// 6 / W: the factor of eq. fb's moving-boundary term 2 w rho0 (u.c) / c_s^2
template <int Q>
__device__ __forceinline__ int rw(int b) { return wint<Q>(b); }
template <int Q>
constexpr double W6 = (double)(WSCALE<Q> / 6);
// 1 / W: a link weight is w_b = rw(b) * WINV exactly, since rw(b) is a power
// of two for every direction a link can take (2, 1; 16, 4, 1)
template <int Q>
constexpr double WINV = 1.0 / WSCALE<Q>;
__device__ __forceinline__ int ropp(int b) { return b == 0 ? 0 : ((b & 1) ? b + 1 : b - 1); }

// q = floor(i / w) and r = i - q w for 0 <= i < 2^31, w >= 1, given
// rw = 1.0 / w: the FP64 product is within 2^-21 of i / w, so its truncation
// is q or one off, and one correction either way makes it exact.  Cheaper
// than an integer division by a value known only at run time.
__device__ __forceinline__ int divmod(int i, int w, double rw, int& r) {
    int q = (int)((double)i * rw);
    r = i - q * w;
    if (r >= w) {
        ++q;
        r -= w;
    } else if (r < 0) {
        --q;
        r += w;
    }
    return q;
}

__device__ __forceinline__ double minimg(double d, int n) {
    if (d >= 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
    return d;
}

// Rotation matrix of q (body -> lab, s_lab = q s_body q^-1).
__device__ __forceinline__ void rotmat(const double q[4], double R[3][3]) {
    const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    R[0][0] = 1 - 2 * (q2 * q2 + q3 * q3);
    R[0][1] = 2 * (q1 * q2 - q0 * q3);
    R[0][2] = 2 * (q1 * q3 + q0 * q2);
    R[1][0] = 2 * (q1 * q2 + q0 * q3);
    R[1][1] = 1 - 2 * (q1 * q1 + q3 * q3);
    R[1][2] = 2 * (q2 * q3 - q0 * q1);
    R[2][0] = 2 * (q1 * q3 - q0 * q2);
    R[2][1] = 2 * (q2 * q3 + q0 * q1);
    R[2][2] = 1 - 2 * (q1 * q1 + q2 * q2);
}

// q(t+1) = exp(Wm / 2) q(t) (eqs. qnplus0, qnplus1): rotation by |Wm| about
// Wm / |Wm|, Wm the mean angular velocity over the step.  With h = |Wm| / 2
// the rotation quaternion is (cos h, (sin h / h) Wm / 2); both are even in h,
// so for h <= 1/4 (every admissible step of a particle with max(a,b,c) >= 1)
// their Taylor series in h^2 up to h^14 give them to rounding (the first
// omitted terms are below 1e-19), without a square root, a division or a
// trigonometric call.
__device__ __forceinline__ void quat_advance(const double q[4], const double Wm[3], double qn[4]) {
    const double h2 = 0.25 * (Wm[0] * Wm[0] + Wm[1] * Wm[1] + Wm[2] * Wm[2]);
    double c, s;  // cos h and sin(h) / h
    if (h2 <= 0.0625) {
        c = 1.0 + h2 * (-1.0 / 2 + h2 * (1.0 / 24 + h2 * (-1.0 / 720 + h2 * (1.0 / 40320 + h2 * (-1.0 / 3628800 +
            h2 * (1.0 / 479001600 + h2 * (-1.0 / 87178291200.0)))))));
        s = 1.0 + h2 * (-1.0 / 6 + h2 * (1.0 / 120 + h2 * (-1.0 / 5040 + h2 * (1.0 / 362880 + h2 * (-1.0 / 39916800 +
            h2 * (1.0 / 6227020800.0 + h2 * (-1.0 / 1307674368000.0)))))));
    } else {
        const double h = sqrt(h2);
        double sn;
        sincos(h, &sn, &c);
        s = sn / h;
    }
    const double t0 = c, t1 = 0.5 * s * Wm[0], t2 = 0.5 * s * Wm[1], t3 = 0.5 * s * Wm[2];
    qn[0] = t0 * q[0] - t1 * q[1] - t2 * q[2] - t3 * q[3];
    qn[1] = t0 * q[1] + t1 * q[0] + t2 * q[3] - t3 * q[2];
    qn[2] = t0 * q[2] - t1 * q[3] + t2 * q[0] + t3 * q[1];
    qn[3] = t0 * q[3] + t1 * q[2] - t2 * q[1] + t3 * q[0];
}

// Symmetric 6x6 solve A x = rhs as A = L D L^T, A in the lower triangle of
// Lw (overwritten by L below the diagonal), one reciprocal per pivot.
// Returns false on a zero pivot.
__device__ __forceinline__ bool ldlt_solve6(double Lw[6][6], double dv[6], double di[6], const double rhs[6],
                                            double sol[6]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double v[6];
#pragma unroll
        for (int k = 0; k < j; ++k) v[k] = Lw[j][k] * dv[k];
        double d = Lw[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lw[j][k] * v[k];
        dv[j] = d;
        ok = ok && fabs(d) > 1e-300;
        di[j] = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double t = Lw[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= Lw[i][k] * v[k];
            Lw[i][j] = t * di[j];
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double t = rhs[i];
#pragma unroll
        for (int k = 0; k < i; ++k) t -= Lw[i][k] * sol[k];
        sol[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) sol[i] *= di[i];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double t = sol[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) t -= Lw[k][i] * sol[k];
        sol[i] = t;
    }
    return ok;
}

// The quadratic form Q of eq. ellipsoidsurface at node (x, y, z); the node is
// solid iff Q < 1.  Body coordinates come from eq. vectrotn with q^-1; the
// operation order is fixed and contraction is off so the decision is
// reproducible bit for bit by any IEEE FP64 evaluation of the same
// expression.
__device__ __forceinline__ double quad_form(const double xc[3], const double q[4], const double ia2[3],
                                            int x, int y, int z, int nx, int ny, int nz) {
#pragma clang fp contract(off)
    const double d0 = minimg((double)x - xc[0], nx);
    const double d1 = minimg((double)y - xc[1], ny);
    const double d2 = minimg((double)z - xc[2], nz);
    const double q0 = q[0], p1 = -q[1], p2 = -q[2], p3 = -q[3];
    const double a0 = (2.0 * q0) * q0 - 1.0;
    const double ps = (p1 * d0 + p2 * d1) + p3 * d2;
    const double c0 = p2 * d2 - p3 * d1;
    const double c1 = p3 * d0 - p1 * d2;
    const double c2 = p1 * d1 - p2 * d0;
    const double u = (a0 * d0 + (2.0 * ps) * p1) + (2.0 * q0) * c0;
    const double v = (a0 * d1 + (2.0 * ps) * p2) + (2.0 * q0) * c1;
    const double w = (a0 * d2 + (2.0 * ps) * p3) + (2.0 * q0) * c2;
    return ((u * u) * ia2[0] + (v * v) * ia2[1]) + (w * w) * ia2[2];
}

// Spheroidal squirmer slip (eq. squirmer) at lab offset d from the centre;
// e = body x axis in the lab frame, a = semi-axis along e, b = the other two.
__device__ __forceinline__ void squirmer_slip(double a, double b, const double e[3], double B1, double B2,
                                              const double d[3], double us[3]) {
    const double z = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
    const double rv0 = d[0] - z * e[0], rv1 = d[1] - z * e[1], rv2 = d[2] - z * e[2];
    const double r = sqrt(rv0 * rv0 + rv1 * rv1 + rv2 * rv2);
    us[0] = us[1] = us[2] = 0.0;
    if (r == 0.0) return;
    const double zc = fmin(fmax(z, -a), a);
    const double eps = sqrt(1.0 - (b * b) / (a * a));
    const double den = sqrt(a * a - eps * eps * zc * zc);
    const double sa = -sqrt(a * a - zc * zc) / den;        // s . e
    const double sr = sqrt(1.0 - eps * eps) * zc / den;   // s . e_perp
    double zeta;
    if (eps > 1e-8)
        zeta = (sqrt(r * r + (z + a * eps) * (z + a * eps)) - sqrt(r * r + (z - a * eps) * (z - a * eps))) /
               (2.0 * a * eps);
    else
        zeta = z / sqrt(r * r + z * z);
    const double k = -sa * (B1 + B2 * zeta);
    const double ir = 1.0 / r;
    us[0] = k * (sa * e[0] + sr * rv0 * ir);
    us[1] = k * (sa * e[1] + sr * rv1 * ir);
    us[2] = k * (sa * e[2] + sr * rv2 * ir);
}

// Whole-wave sums with DPP row shifts and row broadcasts (plain VALU work, no
// LDS traffic): row_shr 1, 2, 4, 8 give inclusive scans of each 16-lane row,
// row_bcast 15 and 31 carry them across rows, so lane 63 ends with the total.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, true);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = dpp_i<CTRL, ROWMASK>(__double2loint(v));
    const int hi = dpp_i<CTRL, ROWMASK>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wsum64(double v) {
    v += dpp_d<0x111, 0xf>(v);
    v += dpp_d<0x112, 0xf>(v);
    v += dpp_d<0x114, 0xf>(v);
    v += dpp_d<0x118, 0xf>(v);
    v += dpp_d<0x142, 0xa>(v);
    v += dpp_d<0x143, 0xc>(v);
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}
__device__ __forceinline__ double wmin64(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wsumi(int v) {
    v += dpp_i<0x111, 0xf>(v);
    v += dpp_i<0x112, 0xf>(v);
    v += dpp_i<0x114, 0xf>(v);
    v += dpp_i<0x118, 0xf>(v);
    v += dpp_i<0x142, 0xa>(v);
    v += dpp_i<0x143, 0xc>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Barrier ordering LDS accesses only: global stores issued before it may
// still be in flight after it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Deterministic block reduction of N doubles; every thread gets the sums.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double (*red)[PWAVES]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = wsum64(v[k]);
        if (lane == 0) red[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0;
        for (int w = 0; w < PWAVES; ++w) s += red[threadIdx.x][w];
        red[threadIdx.x][0] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = red[k][0];
}

// The particle record is read once, cooperatively, into LDS.
__device__ __forceinline__ void stage_particle(const PartDev* P, PartDev* S) {
    static_assert(sizeof(PartDev) % 8 == 0, "PartDev must be a whole number of 8-byte words");
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(P);
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(S);
    for (int k = threadIdx.x; k < (int)(sizeof(PartDev) / 8); k += blockDim.x) dst[k] = src[k];
    __syncthreads();
}

// Where node (x,y,z) keeps its pre-collision population i in the pull
// layout, and what the collide kernel adds when it reads it (wall rows).
template <int Q>
__device__ __forceinline__ void pre_slot(int cv, const BoxDesc& B, double rho0, int i, int x, int y, int z, int& dir,
                                         int& slot, double& add) {
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int sy = wrap(y - rcy(i), ny);
    if (B.walls && rcy(i) != 0 && (sy == 0 || sy == ny - 1)) {
        // off a wall: the node's own f*_opp(i) of the last step plus the wall term
        const double* uw = sy == 0 ? B.wall_lo : B.wall_hi;
        post_slot(cv, ropp(i), x, y, z, nx, ny, nz, dir, slot);
        add = (rw<Q>(i) / W6<Q>) * rho0 * (rcx(i) * uw[0] + rcy(i) * uw[1] + rcz(i) * uw[2]);
    } else {
        pre_slot_open(cv, i, x, y, z, nx, ny, nz, dir, slot);
        add = 0.0;
    }
}

// Element offset (in the box's block) of f*_b at fluid site s: where the
// population a link reads lives in convention cv.
__device__ __forceinline__ long long link_post(int cv, const BoxDesc& B, int b, int s, double rnx, double rny) {
    if (cv == CV_PULL) return (long long)b * B.stride + s;
    if (cv == CV_EVEN) return (long long)ropp(b) * B.stride + s;
    int x, y;
    const int z = divmod(divmod(s, B.nx, rnx, x), B.ny, rny, y);
    return (long long)b * B.stride +
           (wrap(x + rcx(b), B.nx) + B.nx * (wrap(y + rcy(b), B.ny) + B.ny * wrap(z + rcz(b), B.nz)));
}

// Per-thread partial sums of eqs. drag1-drag4 (36 w_b as integers 2 / 1).
template <int Q>
struct ZAcc {
    int cnt6[6];
    int w36s;
    double zfw[9];
    double ztw[6];
    __device__ void clear() {
        for (int k = 0; k < 6; ++k) cnt6[k] = 0;
        w36s = 0;
        for (int k = 0; k < 9; ++k) zfw[k] = 0.0;
        for (int k = 0; k < 6; ++k) ztw[k] = 0.0;
    }
    __device__ __forceinline__ void add(int b, int gx, int gy, int gz, const double xc[3], int nx, int ny, int nz) {
        const int c0 = rcx(b), c1 = rcy(b), c2 = rcz(b), w36 = rw<Q>(b);
        const double r0 = minimg(((double)gx + 0.5 * c0) - xc[0], nx);
        const double r1 = minimg(((double)gy + 0.5 * c1) - xc[1], ny);
        const double r2 = minimg(((double)gz + 0.5 * c2) - xc[2], nz);
        const double rc[3] = {r1 * c2 - r2 * c1, r2 * c0 - r0 * c2, r0 * c1 - r1 * c0};
        const int cc[3] = {c0, c1, c2};
        cnt6[0] += w36 * c0 * c0;
        cnt6[1] += w36 * c0 * c1;
        cnt6[2] += w36 * c0 * c2;
        cnt6[3] += w36 * c1 * c1;
        cnt6[4] += w36 * c1 * c2;
        cnt6[5] += w36 * c2 * c2;
        w36s += w36;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) zfw[3 * ii + jj] += (double)(w36 * cc[ii]) * rc[jj];
        ztw[0] += w36 * rc[0] * rc[0];
        ztw[1] += w36 * rc[0] * rc[1];
        ztw[2] += w36 * rc[0] * rc[2];
        ztw[3] += w36 * rc[1] * rc[1];
        ztw[4] += w36 * rc[1] * rc[2];
        ztw[5] += w36 * rc[2] * rc[2];
    }
};


// Entry (i, j) of zeta (eqs. drag1-drag4) for the particle's link set with
// its centre at xu (unwrapped), from the moments stored when the set was enumerated:
// every link offset is r = rho - d with d = xu - xref, so with D the matrix
// of d x . the blocks are zeta_FU = k Z0, zeta_FW = k (Z1 - Z0 D^T) and
// zeta_TW = k (Z2 - Z1^T D^T - D Z1 + D Z0 D^T), k = rho0 / 6 (36 w = 6 w / c_s^2).
// Both (i, j) and (j, i) evaluate the upper-triangle entry, so the matrix
// stays exactly symmetric.
__device__ __forceinline__ int ut3(int a, int b) {  // upper-triangle index of the symmetric 3x3 (a, b)
    const int l = a < b ? a : b, h = a < b ? b : a;
    return l == 0 ? h : (l == 1 ? 2 + h : 5);
}
// Row j of [d]x (the cross-product matrix of d), for a j known at run time.
__device__ __forceinline__ void cross_row(const double d[3], int j, double r[3]) {
    r[0] = j == 0 ? 0.0 : (j == 1 ? d[2] : -d[1]);
    r[1] = j == 0 ? -d[2] : (j == 1 ? 0.0 : d[0]);
    r[2] = j == 0 ? d[1] : (j == 1 ? -d[0] : 0.0);
}

// zeta of the current link set (eqs. drag1-drag4) at the centre x_u, from
// the moments of the set about x_ref, d = x_u - x_ref.  Lane k < 21 of a
// group: k < 6 an upper entry of zFU (integer sum), k < 15 an entry of zFW
// (zTU = zFW^T), else an upper entry of zTW; each is written to Z[6 i + j]
// and its transposed place.
template <int Q>
__device__ __forceinline__ void zeta_lanes(const PartDev& P, int k, double rho0, double* Z) {
    const double d[3] = {P.xu[0] - P.xref[0], P.xu[1] - P.xref[1], P.xu[2] - P.xref[2]};
    int i, j;
    double v;
    if (k < 6) {
        i = k < 3 ? 0 : (k < 5 ? 1 : 2);
        j = k < 3 ? k : (k < 5 ? k - 2 : 2);
        v = (double)P.zm0[k];
    } else if (k < 15) {
        const int ii = (k - 6) / 3, jj = (k - 6) % 3;
        double D[3];
        cross_row(d, jj, D);
        v = P.zm1[3 * ii + jj];
        for (int b = 0; b < 3; ++b) v -= (double)P.zm0[ut3(ii, b)] * D[b];
        i = ii;
        j = 3 + jj;
    } else {
        const int u = k - 15, ii = u < 3 ? 0 : (u < 5 ? 1 : 2), jj = u < 3 ? u : (u < 5 ? u - 2 : 2);
        double Di[3], Dj[3];
        cross_row(d, ii, Di);
        cross_row(d, jj, Dj);
        v = P.zm2[u];
        for (int b = 0; b < 3; ++b) v -= P.zm1[3 * b + ii] * Dj[b] + Di[b] * P.zm1[3 * b + jj];
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) v += Di[b] * (double)P.zm0[ut3(b, c)] * Dj[c];
        i = 3 + ii;
        j = 3 + jj;
    }
    v = rho0 * v / W6<Q>;
    Z[6 * i + j] = v;
    Z[6 * j + i] = v;
}

// Remap window of a particle: axis-aligned bounding box of the ellipsoid plus
// one node (the whole axis when that is at least the box edge).  It holds
//  - every node inside at t+1: such a node lies beyond x_c - h (h the box
//    half-extent, padded by 1e-9 against the rounding of the inside test),
//  - their fluid neighbours (one node further), and
//  - every node inside at t: a boundary point moves at most half a node per
//    step (the solve keeps |U| + |Omega| max(a,b,c) <= 0.5 and the update
//    uses the mean of two such velocities), so within the same one node.
__device__ __forceinline__ void particle_window(const PartDev& P, const BoxDesc& B, int lo[3], int wn[3],
                                                bool whole[3]) {
    double Rm[3][3];
    rotmat(P.q, Rm);
    const int n3[3] = {B.nx, B.ny, B.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double h = sqrt((Rm[k][0] * P.axes[0]) * (Rm[k][0] * P.axes[0]) +
                              (Rm[k][1] * P.axes[1]) * (Rm[k][1] * P.axes[1]) +
                              (Rm[k][2] * P.axes[2]) * (Rm[k][2] * P.axes[2]));
        lo[k] = (int)floor(P.xc[k] - h - 1e-9) - 1;
        wn[k] = (int)floor(P.xc[k] + h + 1e-9) + 1 - lo[k] + 1;
        whole[k] = wn[k] >= n3[k];
        if (whole[k]) {
            lo[k] = 0;
            wn[k] = n3[k];
        }
    }
}

// Adds every collide-stream block touching the particle's window grown by
// the set's margin to the near set (block-cooperative).
__device__ __forceinline__ void mark_near(const NearSet& ns, const BoxDesc& B, const int wlo[3], const int wwn[3]) {
    const int n3[3] = {B.nx, B.ny, B.nz};
    int lo[3], wn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = wlo[k] - ns.margin;
        wn[k] = wwn[k] + 2 * ns.margin;
        if (wn[k] >= n3[k]) {
            lo[k] = 0;
            wn[k] = n3[k];
        }
    }
    auto add = [&](int blk) {
        if (atomicExch(ns.flags + blk, ns.epoch) != ns.epoch) ns.list[atomicAdd(ns.count, 1)] = blk;
    };
    const int nrows = wn[1] * wn[2];
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
        const int y = wrap(lo[1] + r % wn[1], B.ny), z = wrap(lo[2] + r / wn[1], B.nz);
        const int row = y + B.ny * z;
        if (ns.rows_geom) {
            add(row >> 2);
        } else {
            // x-range [lo0, lo0 + wn0) of this row, split where it wraps
            int xa = wrap(lo[0], B.nx), len = wn[0];
            while (len > 0) {
                const int seg = min(len, B.nx - xa);
                const int s0 = B.nx * row + xa, s1 = s0 + seg - 1;
                for (int t = s0 / TILE; t <= s1 / TILE; ++t) add(B.tile0 + t);
                len -= seg;
                xa = 0;
            }
        }
    }
}

struct SolveShm {
    double red[12][PWAVES];
    double bc[8];
    double Z[36];     // zeta of the current links at x(t)
    double Iblk[9];   // I' + dI/dt
    double IW[3];     // I' Omega(t)
    double rhs[6];    // right-hand side, kept for the predictor-corrector
};

// The links of one thread (l = tid + k PBLOCK, k < KREG): codes and stored
// post-collision populations, held in registers from the force reduction to
// the bounce-back.
template <typename T>
struct LinkRegs {
    uint32_t code[KREG];
    T raw[KREG];
};

// Stages the particle record in LDS (one 8-byte word per thread) and loads
// this thread's links, all from the global record: the record load and the
// code loads go out together, then the population loads, and those stay in
// flight across the LDS write and the barrier.  A lane without a link reads
// element 0 of the box (always valid) and never uses it, so no load sits in
// a branch, where its use, and a wait for it, would follow at once.
template <int ST, int Q>
__device__ __forceinline__ void load_particle(const LaunchPart& a, int p, PartDev* Pl,
                                              LinkRegs<typename Store<ST>::T>& lr) {
    using T = typename Store<ST>::T;
    const PartDev* Pg = a.parts + p;
    constexpr int NW = (int)(sizeof(PartDev) / 8);
    static_assert(sizeof(PartDev) % 8 == 0 && NW <= PBLOCK, "one 8-byte word of the record per thread");
    const int tid = threadIdx.x;
    const unsigned long long sv = tid < NW ? reinterpret_cast<const unsigned long long*>(Pg)[tid] : 0ull;
    const int nl = Pg->nlinks;
    const BoxDesc& B = a.boxes[Pg->box];
    const uint32_t* L = a.links + Pg->lbase;
    const T* f = (const T*)a.f + B.foff;
    const int cv = a.kp.conv;
    const double rnx = 1.0 / B.nx, rny = 1.0 / B.ny;
#pragma unroll
    for (int k = 0; k < KREG; ++k) {
        const int l = tid + k * PBLOCK;
        lr.code[k] = l < nl ? L[l] : 0u;
    }
#pragma unroll
    for (int k = 0; k < KREG; ++k)
        lr.raw[k] = f[link_post(cv, B, (int)(lr.code[k] >> SITE_BITS), (int)(lr.code[k] & SITE_MASK), rnx, rny)];
    if (tid < NW) reinterpret_cast<unsigned long long*>(Pl)[tid] = sv;
    __syncthreads();
}

// Takes a solution of the 6x6 system as U(t+1), Omega(t+1) (bc[0..5], with
// the transition mass per unit link weight in bc[6]), unless a pivot
// vanished, it is not finite, or the surface speed |U| + |Omega| max(a,b,c)
// reaches half a node per step: then the velocities are kept and the
// non-finite flag raised.
__device__ __forceinline__ void accept_solution(const LaunchPart& a, const PartDev& P, bool ok, double sol[6],
                                                const double U0[3], const double W0[3], double* bc) {
    bool bad = !ok;
    for (int k = 0; k < 6; ++k) bad = bad || !isfinite(sol[k]);
    const double amax = fmax(P.axes[0], fmax(P.axes[1], P.axes[2]));
    const double sp = sqrt(sol[0] * sol[0] + sol[1] * sol[1] + sol[2] * sol[2]) +
                      sqrt(sol[3] * sol[3] + sol[4] * sol[4] + sol[5] * sol[5]) * amax;
    bad = bad || !(sp <= 0.5);
    if (bad) {
        atomicOr(a.flags, (int)F_NONFINITE);
        for (int k = 0; k < 6; ++k) sol[k] = k < 3 ? U0[k] : W0[k - 3];
    }
    for (int k = 0; k < 6; ++k) bc[k] = sol[k];
    bc[6] = P.wsum > 0.0 ? P.dm / P.wsum : 0.0;
}

// Steps 3-7 for particle p whose record is staged in LDS (P).  The new state
// goes to global memory; with keep_lds the LDS copy is updated as well.
template <int ST, int Q>
__device__ __forceinline__ void solve_phase(const LaunchPart& a, int p, PartDev& P, SolveShm& sh,
                                            const LinkRegs<typename Store<ST>::T>& lr, bool keep_lds) {
    using S = Store<ST>;
    using T = typename S::T;
    double (*red)[PWAVES] = sh.red;
    double* bc = sh.bc;
    PartDev* Pg = a.parts + p;
    const BoxDesc& B = a.boxes[P.box];
    T* f = (T*)a.f + B.foff;
    const long long st = B.stride;
    const int nx = B.nx, ny = B.ny, nz = B.nz, tid = threadIdx.x;
    // the state at t in registers: with keep_lds the LDS record is
    // overwritten with the state at t+1 while other lanes still need these
    const double xc[3] = {P.xc[0], P.xc[1], P.xc[2]}, xu0[3] = {P.xu[0], P.xu[1], P.xu[2]};
    const double q[4] = {P.q[0], P.q[1], P.q[2], P.q[3]};
    const double B1 = P.B1, B2 = P.B2, ax = P.axes[0], bx = P.axes[1];
    const bool sq = B1 != 0.0 || B2 != 0.0;
    const int nl = P.nlinks;
    const uint32_t* L = a.links + P.lbase;
    const double inv = a.kp.inv_scale, scl = a.kp.scale, rho0 = a.kp.rho0;
    const double rnx = 1.0 / nx, rny = 1.0 / ny;
    double Rm[3][3];
    rotmat(q, Rm);
    const double e[3] = {Rm[0][0], Rm[1][0], Rm[2][0]};

    const uint32_t* code = lr.code;

    // steps 4-5, matrix part, built by the last two waves while the link
    // loads are in flight: zeta of the current link set at x(t) from its
    // moments (three groups of lanes: the zFU, zFW and zTW blocks, each entry
    // also written to its transposed place), and, in one lane, the inertia
    // block I' + dI/dt with I' = R diag(I) R^T and dI/dt = [W]x I' - I' [W]x
    // (W = Omega(t)) or the backward difference I'(t) - I'(t-1), and I' Omega(t)
    const double M = P.M;
    const double U0[3] = {P.U[0], P.U[1], P.U[2]}, W0[3] = {P.W[0], P.W[1], P.W[2]};
    if (tid >= PBLOCK - 64 && tid < PBLOCK - 64 + 21) {
        zeta_lanes<Q>(P, tid - (PBLOCK - 64), rho0, sh.Z);
    } else if (tid == PBLOCK - 128) {
        const double Ib[3] = {P.Ib[0], P.Ib[1], P.Ib[2]};
        double Il[3][3], Id[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Il[i][j] = Rm[i][0] * Ib[0] * Rm[j][0] + Rm[i][1] * Ib[1] * Rm[j][1] + Rm[i][2] * Ib[2] * Rm[j][2];
        if (a.kp.rot == 1) {
            double Rp[3][3];
            rotmat(P.qprev, Rp);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Id[i][j] = Il[i][j] - (Rp[i][0] * Ib[0] * Rp[j][0] + Rp[i][1] * Ib[1] * Rp[j][1] +
                                           Rp[i][2] * Ib[2] * Rp[j][2]);
        } else {
            const double Wx[3][3] = {{0.0, -W0[2], W0[1]}, {W0[2], 0.0, -W0[0]}, {-W0[1], W0[0], 0.0}};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    double d = 0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) d += Wx[i][k] * Il[k][j] - Il[i][k] * Wx[k][j];
                    Id[i][j] = d;
                }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) sh.Iblk[3 * i + j] = Il[i][j] + Id[i][j];
            sh.IW[i] = Il[i][0] * W0[0] + Il[i][1] * W0[1] + Il[i][2] * W0[2];
        }
    }

    // step 3: velocity-independent force and torque, slip part included (the
    // two only ever enter summed).  For the links held in registers (k >= 0)
    // the same pass keeps what the bounce-back needs apart from U(t+1) and
    // Omega(t+1): the slot it writes, r x c, the weight factor and the
    // velocity-independent part of the value (eq. fb: the post-collision
    // population, the transition mass share, the slip term), so that the
    // bounce-back after the solve is a six-term dot product and a store.
    double acc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = 0.0;
    const double dmw = (P.wsum > 0.0 ? P.dm / P.wsum : 0.0) / (double)WSCALE<Q>;
    double bb_base[KREG], bb_kw[KREG], bb_rc[KREG][3];
    long long bb_slot[KREG];
    int bb_b[KREG];
    auto accumulate = [&](uint32_t cd, double fb, int k) {
        const int s = (int)(cd & SITE_MASK), b = (int)(cd >> SITE_BITS);
        int x, y;
        const int z = divmod(divmod(s, nx, rnx, x), ny, rny, y);
        const int c0 = rcx(b), c1 = rcy(b), c2 = rcz(b);
        const double r[3] = {minimg(((double)x + 0.5 * c0) - xc[0], nx), minimg(((double)y + 0.5 * c1) - xc[1], ny),
                             minimg(((double)z + 0.5 * c2) - xc[2], nz)};
        const double rc0 = r[1] * c2 - r[2] * c1, rc1 = r[2] * c0 - r[0] * c2, rc2 = r[0] * c1 - r[1] * c0;
        // eqs. F0, T0 sum the full population f_b = deviation + w_b rho0: the
        // w_b rho0 part cancels over a closed link set, but not where this
        // particle's solid touches another solid or a wall (its links there
        // are missing, and the rest pressure on the exposed side remains)
        const double fb2 = 2.0 * (fb + (rw<Q>(b) * WINV<Q>) * rho0);
        acc[0] += fb2 * c0;
        acc[1] += fb2 * c1;
        acc[2] += fb2 * c2;
        acc[3] += fb2 * rc0;
        acc[4] += fb2 * rc1;
        acc[5] += fb2 * rc2;
        const double kw = (rw<Q>(b) / W6<Q>) * rho0;
        double kuc = 0.0;
        if (sq) {
            double us[3];
            squirmer_slip(ax, bx, e, B1, B2, r, us);
            kuc = kw * (us[0] * c0 + us[1] * c1 + us[2] * c2);
            acc[0] -= kuc * c0;
            acc[1] -= kuc * c1;
            acc[2] -= kuc * c2;
            acc[3] -= kuc * rc0;
            acc[4] -= kuc * rc1;
            acc[5] -= kuc * rc2;
        }
        if (k >= 0) {
            int pd, ps;  // the slot of f_opp(b)(x) the fluid node reads next
            pre_slot_open(a.kp.conv, ropp(b), x, y, z, nx, ny, nz, pd, ps);
            bb_slot[k] = (long long)pd * st + ps;
            bb_base[k] = (fb + dmw * rw<Q>(b)) - kuc;
            bb_kw[k] = kw;
            bb_rc[k][0] = rc0;
            bb_rc[k][1] = rc1;
            bb_rc[k][2] = rc2;
            bb_b[k] = b;
        }
    };
    double fbv[KREG];
#pragma unroll
    for (int k = 0; k < KREG; ++k) fbv[k] = S::cv64(lr.raw[k], inv);
#pragma unroll
    for (int k = 0; k < KREG; ++k)
        if (tid + k * PBLOCK < nl) accumulate(code[k], fbv[k], k);
    // links past the registers (large particles): KOVF per thread per pass,
    // their code loads issued together, then their population loads, then
    // the sums in the same order as one at a time (a lane past the end reads
    // element 0 of the box, always valid, and does not use it)
    for (int l0 = tid + KREG * PBLOCK; l0 < nl; l0 += KOVF * PBLOCK) {
        uint32_t cd[KOVF];
        double fv[KOVF];
#pragma unroll
        for (int j = 0; j < KOVF; ++j) cd[j] = l0 + j * PBLOCK < nl ? L[l0 + j * PBLOCK] : 0u;
#pragma unroll
        for (int j = 0; j < KOVF; ++j)
            fv[j] = S::ld64(f + link_post(a.kp.conv, B, (int)(cd[j] >> SITE_BITS), (int)(cd[j] & SITE_MASK), rnx, rny),
                            inv);
#pragma unroll
        for (int j = 0; j < KOVF; ++j)
            if (l0 + j * PBLOCK < nl) accumulate(cd[j], fv[j], -1);
    }
    block_reduce<6>(acc, red);

    __syncthreads();
    if (tid == 0) {
        // right-hand side [M U + F0' ; I' Omega + T0'] (counter-force density
        // g = -sum F_ext / N on the particle's own nodes, transition impulses)
        double rhs[6];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double gcf = B.gcf[i];  // -fext / (n - n_wall) with the counter-force, else 0
            rhs[i] = M * U0[i] + acc[i] + P.Fext[i] + P.n_solid * gcf + P.Pp[i];
            rhs[3 + i] = sh.IW[i] + acc[3 + i] + P.Text[i] + P.Lp[i];
        }
        // [M + zFU, zFW; zTU, I' + dI/dt + zTW].  The matrix is symmetric
        // (zeta is, I' is, and so are the commutator of [Omega]x with I' and a
        // difference of two inertias), so the elimination runs as A = L D L^T
        // on the lower triangle, in registers.
        double Lw[6][6], dv[6], di[6], sol[6];
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                Lw[i][j] = sh.Z[6 * i + j] + (i >= 3 ? (j >= 3 ? sh.Iblk[3 * (i - 3) + j - 3] : 0.0)
                                                     : (i == j ? M : 0.0));
        const bool ok = ldlt_solve6(Lw, dv, di, rhs, sol);
        if (a.kp.rot == 2) {  // the prediction, checked after the corrector
            for (int i = 0; i < 6; ++i) {
                sh.rhs[i] = rhs[i];
                bc[i] = sol[i];
            }
        } else {
            accept_solution(a, P, ok, sol, U0, W0, bc);
        }
    }
    if (a.kp.rot == 2) {
        // predictor-corrector: the predicted Omega(t+1) rotates q(t) to q*
        // with the mean angular velocity, and the system is solved again with
        // the rotational block zTW + I'(q*) and the same right-hand side
        // (a separate phase, so its registers do not add to the first solve's)
        __syncthreads();
        if (tid == 0) {
            const double Wm[3] = {0.5 * (W0[0] + bc[3]), 0.5 * (W0[1] + bc[4]), 0.5 * (W0[2] + bc[5])};
            double qs[4], Rs[3][3], Lw[6][6], dv[6], di[6], rhs[6], sol[6];
            quat_advance(q, Wm, qs);
            rotmat(qs, Rs);
            const double Ib0 = P.Ib[0], Ib1 = P.Ib[1], Ib2 = P.Ib[2];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                rhs[i] = sh.rhs[i];
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    Lw[i][j] = sh.Z[6 * i + j] + (i >= 3 ? (j >= 3 ? Rs[i - 3][0] * Ib0 * Rs[j - 3][0] +
                                                                         Rs[i - 3][1] * Ib1 * Rs[j - 3][1] +
                                                                         Rs[i - 3][2] * Ib2 * Rs[j - 3][2]
                                                                   : 0.0)
                                                         : (i == j ? M : 0.0));
            }
            const bool ok = ldlt_solve6(Lw, dv, di, rhs, sol);
            accept_solution(a, P, ok, sol, U0, W0, bc);
        }
    }
    __syncthreads();

    // step 7, the hydrodynamic force/torque, position and orientation, spread
    // over three of the upper four waves (one per SIMD), while all waves do
    // the bounce-back (which uses x_c(t), q(t) from registers and U(t+1),
    // Omega(t+1) from bc).  No lane reads an LDS field another lane writes
    // here.  zeta at x(t+1) is evaluated from the link moments when the next
    // step starts.
    static_assert(PBLOCK >= 256, "the state update uses four waves");
    if (tid >= PBLOCK - 64) {
        const int k = tid - (PBLOCK - 64);
        if (k < 6) {  // F, T over the step (eqs. Fsplit, Tsplit)
            const int i = k % 3;
            double z = 0;
            for (int j = 0; j < 6; ++j) z += sh.Z[6 * k + j] * bc[j];
            // each lane clears, after reading it, the pending impulse it used
            if (k < 3) {
                Pg->F[i] = acc[i] + P.Pp[i] - z;
                Pg->Pp[i] = 0.0;
                if (keep_lds) P.Pp[i] = 0.0;
            } else {
                Pg->T[i] = acc[3 + i] + P.Lp[i] - z;
                Pg->Lp[i] = 0.0;
                if (keep_lds) P.Lp[i] = 0.0;
            }
        } else if (k == 6) {
            Pg->dm = 0.0;
            if (keep_lds) P.dm = 0.0;
        }
    } else if (tid >= PBLOCK - 192 && tid < PBLOCK - 192 + 3) {  // position (eq. posupdate), wrapped into the box
        const int i = tid - (PBLOCK - 192);
        const int n3 = i == 0 ? nx : (i == 1 ? ny : nz);
        const double dx = 0.5 * (bc[i] + U0[i]);
        double xn = xc[i] + dx;
        if (xn >= n3) xn -= n3;
        if (xn < 0.0) xn += n3;
        const double xu = xu0[i] + dx;
        Pg->xc[i] = xn;
        Pg->xu[i] = xu;
        Pg->U[i] = bc[i];
        Pg->W[i] = bc[3 + i];
        if (keep_lds) {
            P.xc[i] = xn;
            P.xu[i] = xu;
            P.U[i] = bc[i];
            P.W[i] = bc[3 + i];
        }
    } else if (tid == PBLOCK - 256) {  // orientation (eqs. qnplus0, qnplus1) with the mean angular velocity
        const double Wm[3] = {0.5 * (W0[0] + bc[3]), 0.5 * (W0[1] + bc[4]), 0.5 * (W0[2] + bc[5])};
        double qn[4];
        quat_advance(q, Wm, qn);
        for (int j = 0; j < 4; ++j) {
            Pg->q[j] = qn[j];
            Pg->qprev[j] = q[j];
        }
        if (keep_lds)
            for (int j = 0; j < 4; ++j) {
                P.q[j] = qn[j];
                P.qprev[j] = q[j];
            }
    }

    // step 6: bounce-back into the solid slot the fluid node pulls next step
    const double Un[3] = {bc[0], bc[1], bc[2]}, Wn[3] = {bc[3], bc[4], bc[5]};
    auto bounce = [&](uint32_t cd, double fb) {
        const int s = (int)(cd & SITE_MASK), b = (int)(cd >> SITE_BITS);
        int x, y;
        const int z = divmod(divmod(s, nx, rnx, x), ny, rny, y);
        const int c0 = rcx(b), c1 = rcy(b), c2 = rcz(b);
        const double r[3] = {minimg(((double)x + 0.5 * c0) - xc[0], nx), minimg(((double)y + 0.5 * c1) - xc[1], ny),
                             minimg(((double)z + 0.5 * c2) - xc[2], nz)};
        double ub[3] = {Un[0] + (Wn[1] * r[2] - Wn[2] * r[1]), Un[1] + (Wn[2] * r[0] - Wn[0] * r[2]),
                        Un[2] + (Wn[0] * r[1] - Wn[1] * r[0])};
        if (sq) {
            double us[3];
            squirmer_slip(ax, bx, e, B1, B2, r, us);
            ub[0] += us[0];
            ub[1] += us[1];
            ub[2] += us[2];
        }
        const int w36 = rw<Q>(b);
        const double val = fb - (w36 / W6<Q>) * rho0 * (ub[0] * c0 + ub[1] * c1 + ub[2] * c2) + dmw * w36;
        // the slot of f_opp(b)(x) the fluid node reads next (it comes from the
        // solid node, never off a wall)
        int pd, ps;
        pre_slot_open(a.kp.conv, ropp(b), x, y, z, nx, ny, nz, pd, ps);
        S::st64(f + (long long)pd * st + ps, val, scl);
    };
#pragma unroll
    for (int k = 0; k < KREG; ++k)
        if (tid + k * PBLOCK < nl) {
            // u_b . c = U . c + Omega . (r x c)
            const int b = bb_b[k];
            const double uc = (Un[0] * rcx(b) + Un[1] * rcy(b) + Un[2] * rcz(b)) +
                              (Wn[0] * bb_rc[k][0] + Wn[1] * bb_rc[k][1] + Wn[2] * bb_rc[k][2]);
            S::st64(f + bb_slot[k], bb_base[k] - bb_kw[k] * uc, scl);
        }
    // the links past the registers, KOVF per thread per pass as in the force
    // pass (a link's store never lands on another link's read slot: the
    // store goes to a slot read from the solid side)
    for (int l0 = tid + KREG * PBLOCK; l0 < nl; l0 += KOVF * PBLOCK) {
        uint32_t cd[KOVF];
        double fv[KOVF];
#pragma unroll
        for (int j = 0; j < KOVF; ++j) cd[j] = l0 + j * PBLOCK < nl ? L[l0 + j * PBLOCK] : 0u;
#pragma unroll
        for (int j = 0; j < KOVF; ++j)
            fv[j] = S::ld64(f + link_post(a.kp.conv, B, (int)(cd[j] >> SITE_BITS), (int)(cd[j] & SITE_MASK), rnx, rny),
                            inv);
#pragma unroll
        for (int j = 0; j < KOVF; ++j)
            if (l0 + j * PBLOCK < nl) bounce(cd[j], fv[j]);
    }
}

constexpr int P2B = 8;  // windows of up to P2B chunks of PBLOCK nodes take the batched link pass

struct RemapShm {
    double red[15][PWAVES];
    double mred[PWAVES];
    int wtot[PWAVES];
    int ired[8][PWAVES];
    int wchunk[P2B][PWAVES];  // links per wave and chunk (batched link pass)
};

// Whether the window must be tested again.  At its last test every node of
// the window had |sqrt(Q) - 1| >= smargin / min(a, b, c).  Since then the
// centre moved by dx and the body turned by an angle th: a node x of that
// window then has its body coordinates moved by at most dx + 2 sin(th/2)
// |x - x_c|, which is at most dx + 2 sin(th/2) srho, and sqrt(Q) by at most
// that over min(a, b, c); while that stays below the margin no node of the
// window changed side.  A node outside that window was more than one node
// from the body, and no body point moved by half a node.  Rounding of Q
// (~1e-15) is covered by the 1e-9 allowance.
__device__ __forceinline__ bool scan_needed(const PartDev& P) {
    if (!(P.smargin > 0.0)) return true;
    double dx2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double d = P.xu[k] - P.sref[k];
        dx2 += d * d;
    }
    const double dx = sqrt(dx2);
    // vector part of q conj(qref): its length is sin(th/2)
    const double q0 = P.q[0], r0 = P.qref[0];
    const double v[3] = {P.q[1], P.q[2], P.q[3]}, w[3] = {P.qref[1], P.qref[2], P.qref[3]};
    const double s0 = r0 * v[0] - q0 * w[0] - (v[1] * w[2] - v[2] * w[1]);
    const double s1 = r0 * v[1] - q0 * w[1] - (v[2] * w[0] - v[0] * w[2]);
    const double s2 = r0 * v[2] - q0 * w[2] - (v[0] * w[1] - v[1] * w[0]);
    const double sh = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    const double amax = fmax(P.axes[0], fmax(P.axes[1], P.axes[2]));
    const double dwin = dx + 2.0 * sh * P.srho, dbody = dx + 2.0 * sh * amax;
    return !(dwin * (1.0 + 1e-12) + 1e-9 < P.smargin && dbody < 0.5);
}

// Whether a rescan may test the narrow band of the last full scan only.
// That scan recorded, over its window, every node whose margin was below
// BAND_M (in lattice units; the margin bounds the distance to the surface
// from below); every other node of the box was at least BAND_M from the
// body (nodes outside that window more than one node).  While the body has
// moved by less than BAND_M since (translation plus the rotation's chord over
// that window's radius, shaded for rounding), no node outside the band can
// have changed side.  d0 receives that displacement bound.
__device__ __forceinline__ bool band_ok(const PartDev& P, double& d0) {
    if (!P.bvalid) return false;
    double dx2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double d = P.xu[k] - P.bref[k];
        dx2 += d * d;
    }
    const double dx = sqrt(dx2);
    const double q0 = P.q[0], r0 = P.bqref[0];
    const double v[3] = {P.q[1], P.q[2], P.q[3]}, w[3] = {P.bqref[1], P.bqref[2], P.bqref[3]};
    const double s0 = r0 * v[0] - q0 * w[0] - (v[1] * w[2] - v[2] * w[1]);
    const double s1 = r0 * v[1] - q0 * w[1] - (v[2] * w[0] - v[0] * w[2]);
    const double s2 = r0 * v[2] - q0 * w[2] - (v[0] * w[1] - v[1] * w[0]);
    const double sh = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
    const double amax = fmax(P.axes[0], fmax(P.axes[1], P.axes[2]));
    d0 = dx + 2.0 * sh * P.bsrho;
    return d0 * (1.0 + 1e-12) + 1e-9 < BAND_M * (1.0 - 1e-12) && dx + 2.0 * sh * amax < 0.5;
}

// The remap window of a particle with the reciprocals its index arithmetic
// uses.
struct Win {
    int lo[3], wn[3];
    bool whole[3];
    int nsites;
    double rw0, rw1;
};

// False (and the window flag raised) when the window's bitmask exceeds the
// LDS budget.
__device__ __forceinline__ bool window_of(const LaunchPart& a, const PartDev& P, const BoxDesc& B, Win& w) {
    particle_window(P, B, w.lo, w.wn, w.whole);
    w.nsites = w.wn[0] * w.wn[1] * w.wn[2];
    w.rw0 = 1.0 / w.wn[0];
    w.rw1 = 1.0 / w.wn[1];
    if (((w.nsites + PBLOCK - 1) / PBLOCK) * (PBLOCK / 32) > a.lds_words) {
        if (threadIdx.x == 0) atomicOr(a.flags, (int)F_WINDOW);
        return false;
    }
    return true;
}

// Box coordinates of window node i.
__device__ __forceinline__ void win_node(const Win& w, const BoxDesc& B, int i, int& gx, int& gy, int& gz) {
    int wx, wy;
    const int wz = divmod(divmod(i, w.wn[0], w.rw0, wx), w.wn[1], w.rw1, wy);
    gx = wrap(w.lo[0] + wx, B.nx);
    gy = wrap(w.lo[1] + wy, B.ny);
    gz = wrap(w.lo[2] + wz, B.nz);
}

// Node-map updates that several particles' work-groups may make at once in
// one 32-bit word (two sites): a box's map starts at an even element, so
// site s lies in word s >> 1.  A claim succeeds only on a free (fluid) node.
__device__ __forceinline__ bool claim_node(uint16_t* om, int s, uint16_t me) {
    uint32_t* w = reinterpret_cast<uint32_t*>(om) + (s >> 1);
    const int sh = (s & 1) * 16;
    uint32_t cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
        if ((cur >> sh) & 0xFFFFu) return false;
        const uint32_t prev = atomicCAS(w, cur, cur | ((uint32_t)me << sh));
        if (prev == cur) return true;
        cur = prev;
    }
}
__device__ __forceinline__ void release_node(uint16_t* om, int s) {
    atomicAnd(reinterpret_cast<uint32_t*>(om) + (s >> 1), ~(0xFFFFu << ((s & 1) * 16)));
}

// Marks the cell (8^3 nodes) of a node whose owner changes at this step.
__device__ __forceinline__ void stamp_cell(const LaunchPart& a, const BoxDesc& B, int gx, int gy, int gz,
                                           uint32_t ep) {
    a.stamps[B.coff + (gx >> 3) + B.cnx * ((gy >> 3) + B.cny * (gz >> 3))] = ep;
}

// Whether some node of the window changed owner at this step (a cell of the
// window carries this step's stamp): then links of this particle may have
// appeared or vanished although none of its own nodes changed.  Block-uniform.
__device__ __forceinline__ bool window_stamped(const LaunchPart& a, const BoxDesc& B, const Win& w, uint32_t ep) {
    // per axis up to two runs of coordinates (the window may wrap), as cells
    int c0[3][2], c1[3][2], nr[3], cnt[3];
    const int n3[3] = {B.nx, B.ny, B.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int s0 = w.lo[k], e0 = w.lo[k] + w.wn[k], s1 = 0, e1 = 0;
        if (w.whole[k]) {
            s0 = 0;
            e0 = n3[k];
        } else if (s0 < 0) {
            s1 = 0;
            e1 = e0;
            s0 += n3[k];
            e0 = n3[k];
        } else if (e0 > n3[k]) {
            s1 = 0;
            e1 = e0 - n3[k];
            e0 = n3[k];
        }
        c0[k][0] = s0 >> 3;
        c1[k][0] = (e0 - 1) >> 3;
        nr[k] = e1 > s1 ? 2 : 1;
        c0[k][1] = s1 >> 3;
        c1[k][1] = e1 > s1 ? (e1 - 1) >> 3 : -1;
        cnt[k] = (c1[k][0] - c0[k][0] + 1) + (nr[k] == 2 ? c1[k][1] - c0[k][1] + 1 : 0);
    }
    auto cell = [&](int k, int j) {
        const int n0 = c1[k][0] - c0[k][0] + 1;
        return j < n0 ? c0[k][0] + j : c0[k][1] + (j - n0);
    };
    bool hit = false;
    const int total = cnt[0] * cnt[1] * cnt[2];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int jx = t % cnt[0], jy = (t / cnt[0]) % cnt[1], jz = t / (cnt[0] * cnt[1]);
        const int c = cell(0, jx) + B.cnx * (cell(1, jy) + B.cny * cell(2, jz));
        hit = hit || a.stamps[B.coff + c] == ep;
    }
    return __syncthreads_or(hit) != 0;
}

// Pass 1 of the remap over the window: the solid test of eq. ellipsoidsurface
// at the particle's new pose.
//  mode 0 (step): a node of this particle no longer inside is uncovered: it
//    gets f = f_eq(rho0, U + W x r) and its momentum is paid by the particle
//    (reading R9); a node inside that is not yet this particle's is a
//    candidate, claimed afterwards by claim_pass (so that, with several
//    particles in a box, every release is done before any claim);
//  mode 1 (add): every node inside is a candidate, no book-keeping;
//  mode 2 (remove): every node of this particle is released.
// bits (LDS; may be null): this particle's nodes after the step.  cand: the
// candidate bits (LDS, or this particle's global area).  With ep != 0 the
// cells of released and candidate nodes are stamped.  Also records the skip
// test's reference (pose, margin, window radius), and with mode 0 the pending
// mass / momentum / angular momentum and the solid count.  Returns bit 0 set
// when some node was released or is a candidate, bit 1 when some node is a
// candidate; block-uniform.
template <int ST, int Q>
__device__ __forceinline__ int scan_pass(const LaunchPart& a, int p, PartDev& P, const BoxDesc& B, const Win& w, uint32_t* bits,
                         uint32_t* cand, RemapShm& sh, uint32_t ep) {
    using S = Store<ST>;
    using T = typename S::T;
    double (*red)[PWAVES] = sh.red;
    int (*ired)[PWAVES] = sh.ired;
    PartDev* Pg = a.parts + p;
    T* f = (T*)a.f + B.foff;
    uint16_t* om = a.omap + B.ooff;
    const long long st = B.stride;
    const int nx = B.nx, ny = B.ny, nz = B.nz, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const uint16_t me = (uint16_t)(p + 1);
    const int mode = a.mode;
    const double xc[3] = {P.xc[0], P.xc[1], P.xc[2]};
    const double q[4] = {P.q[0], P.q[1], P.q[2], P.q[3]};
    const double ia2[3] = {P.ia2[0], P.ia2[1], P.ia2[2]};
    const double U[3] = {P.U[0], P.U[1], P.U[2]}, W[3] = {P.W[0], P.W[1], P.W[2]};
    const double scl = a.kp.scale, rho0 = a.kp.rho0;
    const int nsites = w.nsites;

    double tacc[7] = {0, 0, 0, 0, 0, 0, 0};
    double mloc = 1.0;  // lower bound of |sqrt(Q) - 1| over this thread's nodes
    int nsol = 0;
    bool released = false, candidate = false;
    // the narrow band of this scan (mode 0 and 1): window nodes whose margin
    // is below BAND_M
    const bool rec_band = a.use_band && mode != 2;
    uint32_t* bandw = a.band + (size_t)p * a.lds_words;
    const double band_q = BAND_M / fmin(P.axes[0], fmin(P.axes[1], P.axes[2]));
    for (int base = 0; base < nsites; base += PBLOCK * KSCAN) {
        uint16_t own[KSCAN];
        int sidx[KSCAN], gxyz[KSCAN][3];
#pragma unroll
        for (int k = 0; k < KSCAN; ++k) {  // issue the node-map loads of the whole group first
            const int i = base + k * PBLOCK + tid;
            sidx[k] = -1;
            own[k] = 0;
            if (i < nsites) {
                win_node(w, B, i, gxyz[k][0], gxyz[k][1], gxyz[k][2]);
                sidx[k] = gxyz[k][0] + nx * (gxyz[k][1] + ny * gxyz[k][2]);
                own[k] = om[sidx[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < KSCAN; ++k) {
            if (base + k * PBLOCK >= nsites) break;  // uniform over the block
            bool in = false, cd = false, bnd = false;
            const int s = sidx[k];
            if (s >= 0) {
                const int gx = gxyz[k][0], gy = gxyz[k][1], gz = gxyz[k][2];
                if (mode == 2) {
                    if (own[k] == me) {
                        release_node(om, s);
                        released = true;
                    }
                } else {
                    const double Qv = quad_form(xc, q, ia2, gx, gy, gz, nx, ny, nz);
                    in = Qv < 1.0;
                    // sqrt(Q) <= (Q + 1) / 2, so |sqrt(Q) - 1| = |Q - 1| / (sqrt(Q) + 1) >= 2 |Q - 1| / (Q + 3)
                    const double mq = 2.0 * fabs(Qv - 1.0) / (Qv + 3.0);
                    mloc = fmin(mloc, mq);
                    bnd = mq < band_q;
                    if (in && own[k] == 0xFFFFu) {  // a wall node
                        atomicOr(a.flags, (int)F_OVERLAP);
                        in = false;
                    }
                    if (in && own[k] != me) {
                        cd = true;
                        candidate = true;
                        if (ep) stamp_cell(a, B, gx, gy, gz, ep);
                    } else if (!in && own[k] == me) {
                        released = true;
                        if (ep) stamp_cell(a, B, gx, gy, gz, ep);
                        if (mode == 0) {
                            // uncovered: f = f_eq(rho0, U + W x r), paid by the particle
                            const double r[3] = {minimg((double)gx - xc[0], nx), minimg((double)gy - xc[1], ny),
                                                 minimg((double)gz - xc[2], nz)};
                            const double u[3] = {U[0] + (W[1] * r[2] - W[2] * r[1]),
                                                 U[1] + (W[2] * r[0] - W[0] * r[2]),
                                                 U[2] + (W[0] * r[1] - W[1] * r[0])};
                            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                            for (int j = 0; j < Q; ++j) {
                                int dir, slot;
                                double add;
                                pre_slot<Q>(a.kp.conv, B, rho0, j, gx, gy, gz, dir, slot, add);
                                const double cu = rcx(j) * u[0] + rcy(j) * u[1] + rcz(j) * u[2];
                                const double dev = (rw<Q>(j) / (double)WSCALE<Q>) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                                S::st64(f + (long long)dir * st + slot, dev - add, scl);
                            }
                            // the new node holds rho0: no excess mass
                            const double pu[3] = {rho0 * u[0], rho0 * u[1], rho0 * u[2]};
                            tacc[1] -= pu[0];
                            tacc[2] -= pu[1];
                            tacc[3] -= pu[2];
                            tacc[4] -= r[1] * pu[2] - r[2] * pu[1];
                            tacc[5] -= r[2] * pu[0] - r[0] * pu[2];
                            tacc[6] -= r[0] * pu[1] - r[1] * pu[0];
                        }
                        release_node(om, s);
                    }
                    nsol += in ? 1 : 0;
                }
            }
            const int w0 = (base + k * PBLOCK + wv * 64) >> 5;
            const unsigned long long cm = __ballot(cd);
            if (lane == 0) {
                cand[w0] = (uint32_t)cm;
                cand[w0 + 1] = (uint32_t)(cm >> 32);
            }
            if (bits) {
                const unsigned long long m = __ballot(in);
                if (lane == 0) {
                    bits[w0] = (uint32_t)m;
                    bits[w0 + 1] = (uint32_t)(m >> 32);
                }
            }
            if (rec_band) {
                const unsigned long long m = __ballot(bnd);
                if (lane == 0) {
                    bandw[w0] = (uint32_t)m;
                    bandw[w0 + 1] = (uint32_t)(m >> 32);
                }
            }
        }
    }
    if (mode != 2) {
        const double wm = wmin64(mloc);
        if (lane == 0) sh.mred[wv] = wm;
    }
    const bool anycand = __syncthreads_or(candidate) != 0;
    const bool changed = anycand || __syncthreads_or(released) != 0;

    if (mode != 2 && tid < 9) {
        // the reference of the skip test: this pose, and the margin in
        // distance units (sqrt(Q) is 1 / min(a, b, c)-Lipschitz in the body
        // coordinates), shaded down for rounding
        if (tid == 0) {
            double m = sh.mred[0];
            for (int v = 1; v < PWAVES; ++v) m = fmin(m, sh.mred[v]);
            const double amin = fmin(P.axes[0], fmin(P.axes[1], P.axes[2]));
            Pg->smargin = m * amin * (1.0 - 1e-12);
        } else if (tid < 4) {
            Pg->sref[tid - 1] = P.xu[tid - 1];
        } else if (tid < 8) {
            Pg->qref[tid - 4] = P.q[tid - 4];
        } else {
            // largest |x - x_c| over the window's nodes
            const int n3[3] = {nx, ny, nz};
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double e = w.whole[k] ? 0.5 * n3[k]
                                            : fmax(xc[k] - w.lo[k], (double)(w.lo[k] + w.wn[k] - 1) - xc[k]);
                r2 += e * e;
            }
            Pg->srho = sqrt(r2);
            // the band's reference: this pose, this window and its radius
            if (rec_band) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Pg->bref[k] = P.xu[k];
                    Pg->blo[k] = w.lo[k];
                    Pg->bwn[k] = w.wn[k];
                }
                for (int k = 0; k < 4; ++k) Pg->bqref[k] = P.q[k];
                Pg->bsrho = sqrt(r2);
            }
            Pg->bvalid = rec_band ? 1 : 0;
        }
    }
    if (mode == 2 && tid == 0) Pg->bvalid = 0;
    if (changed) {
        // solid count and (mode 0) the uncovered nodes' book-keeping
        if (mode == 0) block_reduce<7>(tacc, red);
        const int sm = wsumi(nsol);
        if (lane == 0) ired[7][wv] = sm;
        __syncthreads();
        // one lane per output; each reads and rewrites only its own field of
        // the LDS copy, which the claims then start from
        if (tid == 44) {
            int ns = 0;
            for (int v = 0; v < PWAVES; ++v) ns += ired[7][v];
            if (ns != P.n_solid) atomicAdd(&a.rt[P.box].n_solid, ns - P.n_solid);
            Pg->n_solid = ns;
            P.n_solid = ns;
        } else if (mode == 0 && tid >= 37 && tid < 44) {
            const int k = tid - 37;  // dm, Pp[3], Lp[3]
            double* fld = k == 0 ? &P.dm : (k < 4 ? &P.Pp[k - 1] : &P.Lp[k - 4]);
            double* gfld = k == 0 ? &Pg->dm : (k < 4 ? &Pg->Pp[k - 1] : &Pg->Lp[k - 4]);
            const double nv = *fld + tacc[k];
            *gfld = nv;
            *fld = nv;
        }
        __syncthreads();
    }
    return (changed ? 1 : 0) | (anycand ? 2 : 0);
}

// This particle's nodes over the window, as window bits, from the node map.
__device__ __forceinline__ void bits_from_map(const LaunchPart& a, int p, const BoxDesc& B, const Win& w, uint32_t* bits) {
    const uint16_t* om = a.omap + B.ooff;
    const uint16_t me = (uint16_t)(p + 1);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int base = 0; base < w.nsites; base += PBLOCK * KSCAN) {
        bool in[KSCAN];
#pragma unroll
        for (int k = 0; k < KSCAN; ++k) {
            const int i = base + k * PBLOCK + tid;
            in[k] = false;
            if (i < w.nsites) {
                int gx, gy, gz;
                win_node(w, B, i, gx, gy, gz);
                in[k] = om[gx + B.nx * (gy + B.ny * gz)] == me;
            }
        }
#pragma unroll
        for (int k = 0; k < KSCAN; ++k) {
            if (base + k * PBLOCK >= w.nsites) break;  // uniform over the block
            const unsigned long long m = __ballot(in[k]);
            if (lane == 0) {
                const int w0 = (base + k * PBLOCK + wv * 64) >> 5;
                bits[w0] = (uint32_t)m;
                bits[w0 + 1] = (uint32_t)(m >> 32);
            }
        }
    }
    __syncthreads();
}

// LDS words of the particle kernels' dynamic area (window bitmask and link
// stage), which the band's list may fill.
__host__ __device__ constexpr int band_list_cap(int lds_words) { return lds_words + (lds_words > STAGE ? lds_words : STAGE); }

// The band's nodes (indices in the window of its full scan), in index
// order, into list[0, nb) (LDS, cap entries): a block-wide prefix over the
// band's bit words.  False, with nb the count, when they do not fit.
__device__ __forceinline__ bool band_list(const uint32_t* bandw, int nwords, uint32_t* list, int cap,
                                          RemapShm& sh, int& nb) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int per = (nwords + PBLOCK - 1) / PBLOCK;  // consecutive words per thread
    int cnt = 0;
    for (int j = 0; j < per; ++j) {
        const int wi = tid * per + j;
        if (wi < nwords) cnt += __popc(bandw[wi]);
    }
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh.wtot[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int v = 0; v < PWAVES; ++v) {
        const int t = sh.wtot[v];
        if (v < wv) before += t;
        total += t;
    }
    nb = total;
    if (total > cap) {  // uniform over the block
        __syncthreads();
        return false;
    }
    int off = before + incl - cnt;
    for (int j = 0; j < per; ++j) {
        const int wi = tid * per + j;
        if (wi < nwords) {
            uint32_t m = bandw[wi];
            while (m) {
                const int bt = __ffs(m) - 1;
                m &= m - 1;
                list[off++] = (uint32_t)(wi * 32 + bt);
            }
        }
    }
    __syncthreads();
    return true;
}

// Pass 1 over the narrow band of the last full scan only (mode 0, when
// band_ok holds; d0 its displacement bound).  Every node outside the band
// keeps its side (band_ok), so the outcome equals scan_pass's: the same
// releases and uncovered-node book-keeping, the same candidates (cand, over
// the current window), the same solid count, and with bits (LDS; the fused
// path) this particle's nodes after the step.  The band's nodes are first
// tested without side effects (listed in index order in lst, cap entries of
// LDS that the pass may overwrite, when they fit); only if some node changes
// side are the candidate bits cleared, bits read from the node map (before
// any change) and the changes made.  The skip test's reference becomes this
// pose, with the margin of the band's nodes here and BAND_M - d0 for every
// other node.  Returns as scan_pass.
template <int ST, int Q>
__device__ __forceinline__ int band_pass(const LaunchPart& a, int p, PartDev& P, const BoxDesc& B, const Win& w,
                                         uint32_t* bits, uint32_t* cand, uint32_t* lst, int cap, RemapShm& sh,
                                         uint32_t ep, double d0) {
    using S = Store<ST>;
    double (*red)[PWAVES] = sh.red;
    int (*ired)[PWAVES] = sh.ired;
    PartDev* Pg = a.parts + p;
    auto* f = (typename S::T*)a.f + B.foff;
    uint16_t* om = a.omap + B.ooff;
    const long long st = B.stride;
    const int nx = B.nx, ny = B.ny, nz = B.nz, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const uint16_t me = (uint16_t)(p + 1);
    const double xc[3] = {P.xc[0], P.xc[1], P.xc[2]};
    const double q[4] = {P.q[0], P.q[1], P.q[2], P.q[3]};
    const double ia2[3] = {P.ia2[0], P.ia2[1], P.ia2[2]};
    const double U[3] = {P.U[0], P.U[1], P.U[2]}, W[3] = {P.W[0], P.W[1], P.W[2]};
    const double scl = a.kp.scale, rho0 = a.kp.rho0;
    // the window of the full scan the band belongs to
    Win w0;
    w0.lo[0] = P.blo[0];
    w0.lo[1] = P.blo[1];
    w0.lo[2] = P.blo[2];
    w0.wn[0] = P.bwn[0];
    w0.wn[1] = P.bwn[1];
    w0.wn[2] = P.bwn[2];
    w0.whole[0] = w0.wn[0] >= nx;
    w0.whole[1] = w0.wn[1] >= ny;
    w0.whole[2] = w0.wn[2] >= nz;
    w0.nsites = w0.wn[0] * w0.wn[1] * w0.wn[2];
    w0.rw0 = 1.0 / w0.wn[0];
    w0.rw1 = 1.0 / w0.wn[1];
    const uint32_t* bandw = a.band + (size_t)p * a.lds_words;
    const int bwords = (w0.nsites + 31) >> 5;
    int nb = 0;
    const bool listed = lst && band_list(bandw, bwords, lst, cap, sh, nb);

    // visits the band's nodes that lie in the current window, the node-map
    // loads of KSCAN nodes per thread in flight together: fn(gx, gy, gz, s, i1, own)
    auto visit = [&](bool from_list, auto&& fn) {
        const int n = from_list ? nb : w0.nsites;
        for (int base = 0; base < n; base += PBLOCK * KSCAN) {
            uint16_t own[KSCAN];
            int sidx[KSCAN], widx[KSCAN], gxyz[KSCAN][3];
#pragma unroll
            for (int k = 0; k < KSCAN; ++k) {
                const int j = base + k * PBLOCK + tid;
                sidx[k] = -1;
                widx[k] = -1;
                own[k] = 0;
                int i = -1;
                if (j < n) i = from_list ? (int)lst[j] : (((bandw[j >> 5] >> (j & 31)) & 1u) ? j : -1);
                if (i >= 0) {
                    win_node(w0, B, i, gxyz[k][0], gxyz[k][1], gxyz[k][2]);
                    // its index in the current window (a band node outside it is
                    // more than a node from the body: it stays fluid)
                    const int ox = w.whole[0] ? gxyz[k][0] : wrap(gxyz[k][0] - w.lo[0], nx);
                    const int oy = w.whole[1] ? gxyz[k][1] : wrap(gxyz[k][1] - w.lo[1], ny);
                    const int oz = w.whole[2] ? gxyz[k][2] : wrap(gxyz[k][2] - w.lo[2], nz);
                    if (ox < w.wn[0] && oy < w.wn[1] && oz < w.wn[2]) {
                        widx[k] = ox + w.wn[0] * (oy + w.wn[1] * oz);
                        sidx[k] = gxyz[k][0] + nx * (gxyz[k][1] + ny * gxyz[k][2]);
                        own[k] = om[sidx[k]];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < KSCAN; ++k)
                if (sidx[k] >= 0) fn(gxyz[k][0], gxyz[k][1], gxyz[k][2], sidx[k], widx[k], own[k]);
        }
    };

    // test: the margins, and whether any node changes side
    double mloc = 1.0;
    bool chg = false;
    visit(listed, [&](int gx, int gy, int gz, int s, int i1, uint16_t own) {
        const double Qv = quad_form(xc, q, ia2, gx, gy, gz, nx, ny, nz);
        mloc = fmin(mloc, 2.0 * fabs(Qv - 1.0) / (Qv + 3.0));
        const bool in = Qv < 1.0;
        chg = chg || (in ? own != me : own == me);
    });
    {
        const double wm = wmin64(mloc);
        if (lane == 0) sh.mred[wv] = wm;
    }
    const bool any = __syncthreads_or(chg) != 0;
    if (tid < 9) {
        if (tid == 0) {
            double m = sh.mred[0];
            for (int v = 1; v < PWAVES; ++v) m = fmin(m, sh.mred[v]);
            const double amin = fmin(P.axes[0], fmin(P.axes[1], P.axes[2]));
            Pg->smargin = fmin(m * amin, BAND_M - d0) * (1.0 - 1e-12);
        } else if (tid < 4) {
            Pg->sref[tid - 1] = P.xu[tid - 1];
        } else if (tid < 8) {
            Pg->qref[tid - 4] = P.q[tid - 4];
        } else {
            const int n3[3] = {nx, ny, nz};
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double e = w.whole[k] ? 0.5 * n3[k]
                                            : fmax(xc[k] - w.lo[k], (double)(w.lo[k] + w.wn[k] - 1) - xc[k]);
                r2 += e * e;
            }
            Pg->srho = sqrt(r2);
        }
    }
    if (!any) return 0;

    // some node changes side: candidate bits over the current window, this
    // particle's nodes from the map before any change (fused path), then the
    // changes, as scan_pass makes them
    const int nwords = (w.nsites + 31) >> 5;
    for (int j = tid; j < nwords; j += PBLOCK) cand[j] = 0u;
    const bool relist = listed && !bits;  // bits overwrites the LDS the list is in
    if (bits) bits_from_map(a, p, B, w, bits);  // ends with a barrier
    else __syncthreads();
    double tacc[7] = {0, 0, 0, 0, 0, 0, 0};
    int dsol = 0;  // change of the solid count
    bool released = false, candidate = false;
    visit(relist, [&](int gx, int gy, int gz, int s, int i1, uint16_t own) {
        const double Qv = quad_form(xc, q, ia2, gx, gy, gz, nx, ny, nz);
        bool in = Qv < 1.0;
        if (in && own == 0xFFFFu) {  // a wall node
            atomicOr(a.flags, (int)F_OVERLAP);
            in = false;
        }
        if (in && own != me) {
            candidate = true;
            atomicOr(&cand[i1 >> 5], 1u << (i1 & 31));
            if (bits) atomicOr(&bits[i1 >> 5], 1u << (i1 & 31));
            if (ep) stamp_cell(a, B, gx, gy, gz, ep);
            ++dsol;
        } else if (!in && own == me) {
            released = true;
            if (bits) atomicAnd(&bits[i1 >> 5], ~(1u << (i1 & 31)));
            if (ep) stamp_cell(a, B, gx, gy, gz, ep);
            --dsol;
            // uncovered: f = f_eq(rho0, U + W x r), paid by the particle
            const double r[3] = {minimg((double)gx - xc[0], nx), minimg((double)gy - xc[1], ny),
                                 minimg((double)gz - xc[2], nz)};
            const double u[3] = {U[0] + (W[1] * r[2] - W[2] * r[1]), U[1] + (W[2] * r[0] - W[0] * r[2]),
                                 U[2] + (W[0] * r[1] - W[1] * r[0])};
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            for (int j = 0; j < Q; ++j) {
                int dir, slot;
                double add;
                pre_slot<Q>(a.kp.conv, B, rho0, j, gx, gy, gz, dir, slot, add);
                const double cu = rcx(j) * u[0] + rcy(j) * u[1] + rcz(j) * u[2];
                const double dev = (rw<Q>(j) / (double)WSCALE<Q>) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                S::st64(f + (long long)dir * st + slot, dev - add, scl);
            }
            const double pu[3] = {rho0 * u[0], rho0 * u[1], rho0 * u[2]};
            tacc[1] -= pu[0];
            tacc[2] -= pu[1];
            tacc[3] -= pu[2];
            tacc[4] -= r[1] * pu[2] - r[2] * pu[1];
            tacc[5] -= r[2] * pu[0] - r[0] * pu[2];
            tacc[6] -= r[0] * pu[1] - r[1] * pu[0];
            release_node(om, s);
        }
    });
    const bool anycand = __syncthreads_or(candidate) != 0;
    const bool changed = anycand || __syncthreads_or(released) != 0;
    if (changed) {
        block_reduce<7>(tacc, red);
        const int sm = wsumi(dsol);
        if (lane == 0) ired[7][wv] = sm;
        __syncthreads();
        if (tid == 44) {
            int ds = 0;
            for (int v = 0; v < PWAVES; ++v) ds += ired[7][v];
            const int ns = P.n_solid + ds;
            if (ns != P.n_solid) atomicAdd(&a.rt[P.box].n_solid, ns - P.n_solid);
            Pg->n_solid = ns;
            P.n_solid = ns;
        } else if (tid >= 37 && tid < 44) {
            const int k = tid - 37;  // dm, Pp[3], Lp[3]
            double* fld = k == 0 ? &P.dm : (k < 4 ? &P.Pp[k - 1] : &P.Lp[k - 4]);
            double* gfld = k == 0 ? &Pg->dm : (k < 4 ? &Pg->Pp[k - 1] : &Pg->Lp[k - 4]);
            const double nv = *fld + tacc[k];
            *gfld = nv;
            *fld = nv;
        }
        __syncthreads();
    }
    return (changed ? 1 : 0) | (anycand ? 2 : 0);
}

// Claims the candidate nodes of pass 1 (cand: bits over the window, in LDS or
// global memory).  Window node i is claimed by thread i mod PBLOCK, as in
// pass 1 (neighbouring surface nodes, which change side together, go to
// different threads), so the sums below do not depend on where the bits
// are held.  A node another particle or a wall holds is an overlap.  Mode 0: a covered node's momentum
// and its mass in excess of rho0 go to the particle, its angular momentum
// about x_c(t+1) (reading R9); the populations it holds are read after every
// bounce-back and release of the step.
template <int ST, int Q>
__device__ __forceinline__ void claim_pass(const LaunchPart& a, int p, PartDev& P, const BoxDesc& B, const Win& w,
                           const uint32_t* cand, RemapShm& sh) {
    using S = Store<ST>;
    using T = typename S::T;
    const T* f = (const T*)a.f + B.foff;
    uint16_t* om = a.omap + B.ooff;
    PartDev* Pg = a.parts + p;
    const long long st = B.stride;
    const int nx = B.nx, ny = B.ny, nz = B.nz, tid = threadIdx.x;
    const uint16_t me = (uint16_t)(p + 1);
    const double xc[3] = {P.xc[0], P.xc[1], P.xc[2]};
    const double inv = a.kp.inv_scale, rho0 = a.kp.rho0;
    double tacc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int base = 0; base < w.nsites; base += PBLOCK) {
        const int i = base + tid;
        // a wave reads two bit words, each shared by 32 lanes
        if (i >= w.nsites || !((cand[i >> 5] >> (i & 31)) & 1u)) continue;
        {
            int gx, gy, gz;
            win_node(w, B, i, gx, gy, gz);
            const int s = gx + nx * (gy + ny * gz);
            if (!claim_node(om, s, me)) {
                atomicOr(a.flags, (int)F_OVERLAP);
                continue;
            }
            if (a.mode != 0) continue;
            const double r[3] = {minimg((double)gx - xc[0], nx), minimg((double)gy - xc[1], ny),
                                 minimg((double)gz - xc[2], nz)};
            double mm = 0, pm[3] = {0, 0, 0};
            // unrolled, so that the Q loads are in flight together
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                int dir, slot;
                double add;
                pre_slot<Q>(a.kp.conv, B, rho0, j, gx, gy, gz, dir, slot, add);
                const double v = S::ld64(f + (long long)dir * st + slot, inv) + add;
                mm += v;
                pm[0] += rcx(j) * v;
                pm[1] += rcy(j) * v;
                pm[2] += rcz(j) * v;
            }
            tacc[0] += mm;
            tacc[1] += pm[0];
            tacc[2] += pm[1];
            tacc[3] += pm[2];
            tacc[4] += r[1] * pm[2] - r[2] * pm[1];
            tacc[5] += r[2] * pm[0] - r[0] * pm[2];
            tacc[6] += r[0] * pm[1] - r[1] * pm[0];
        }
    }
    if (a.mode != 0) {
        __syncthreads();
        return;
    }
    block_reduce<7>(tacc, sh.red);
    if (tid >= 37 && tid < 44) {
        const int k = tid - 37;  // dm, Pp[3], Lp[3], added to the uncovered nodes' sums of pass 1
        if (k == 0) Pg->dm = P.dm + tacc[0];
        else if (k < 4) Pg->Pp[k - 1] = P.Pp[k - 1] + tacc[k];
        else Pg->Lp[k - 4] = P.Lp[k - 4] + tacc[k];
    }
    __syncthreads();
}


// Pass 2: the boundary links (fluid x, x + c_b solid of this particle; bits
// holds this particle's nodes over the window), staged in LDS and written in
// (window index, direction) order, and their moments, from which zeta of
// eqs. drag1-drag4 is evaluated when the next step starts.
template <int Q>
__device__ __forceinline__ void link_pass(const LaunchPart& a, int p, const PartDev& P, const BoxDesc& B, const Win& w,
                          const uint32_t* bits, uint32_t* stage, RemapShm& sh) {
    double (*red)[PWAVES] = sh.red;
    int* wtot = sh.wtot;
    int (*ired)[PWAVES] = sh.ired;
    PartDev* Pg = a.parts + p;
    const uint16_t* om = a.omap + B.ooff;
    const int nx = B.nx, ny = B.ny, nz = B.nz, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const double xc[3] = {P.xc[0], P.xc[1], P.xc[2]};
    const int nsites = w.nsites;
    const int* lo = w.lo;
    const int* wn = w.wn;
    const bool* whole = w.whole;
    const double rw0 = w.rw0, rw1 = w.rw1;

    ZAcc<Q> z;
    z.clear();
    int running = 0;
    const int lcap = P.lcap;
    uint32_t* L = a.links + P.lbase;
    // the link mask of window node i: bit b set when i is fluid and i + c_b
    // is solid here (the node map is read only where bits[] says not this
    // particle's)
    auto link_mask = [&](int i, uint16_t own, int& s, int& gx, int& gy, int& gz) -> uint32_t {
        uint32_t lm = 0;
        int wx, wy;
        const int wz = divmod(divmod(i, wn[0], rw0, wx), wn[1], rw1, wy);
        gx = wrap(lo[0] + wx, nx);
        gy = wrap(lo[1] + wy, ny);
        gz = wrap(lo[2] + wz, nz);
        s = gx + nx * (gy + ny * gz);
        if (own == 0) {
#pragma unroll
            for (int b = 1; b < Q; ++b) {
                int nwx = wx + cx(b), nwy = wy + cy(b), nwz = wz + cz(b);
                if (whole[0]) nwx = wrap(nwx, wn[0]);
                else if (nwx < 0 || nwx >= wn[0]) continue;
                if (whole[1]) nwy = wrap(nwy, wn[1]);
                else if (nwy < 0 || nwy >= wn[1]) continue;
                if (whole[2]) nwz = wrap(nwz, wn[2]);
                else if (nwz < 0 || nwz >= wn[2]) continue;
                const int ni = nwx + wn[0] * (nwy + wn[1] * nwz);
                if ((bits[ni >> 5] >> (ni & 31)) & 1u) lm |= 1u << b;
            }
        }
        return lm;
    };
    const int nch = (nsites + PBLOCK - 1) / PBLOCK;
    if (nch <= P2B) {
        // small windows: every chunk's masks first (the node-map loads of all
        // chunks in flight together), one block scan over all chunks, one
        // staged copy-out; same order and same sums as below
        uint32_t lmv[P2B];
        int sv[P2B], offv[P2B];
        uint16_t ownv[P2B];
#pragma unroll
        for (int c = 0; c < P2B; ++c) {
            const int i = c * PBLOCK + tid;
            ownv[c] = 1;  // not fluid
            if (i < nsites && !((bits[i >> 5] >> (i & 31)) & 1u)) {
                int wx, wy;
                const int wz = divmod(divmod(i, wn[0], rw0, wx), wn[1], rw1, wy);
                ownv[c] = om[wrap(lo[0] + wx, nx) + nx * (wrap(lo[1] + wy, ny) + ny * wrap(lo[2] + wz, nz))];
            }
        }
#pragma unroll
        for (int c = 0; c < P2B; ++c) {
            lmv[c] = 0;
            sv[c] = 0;
            offv[c] = 0;
            if (c < nch) {  // uniform over the block
                const int i = c * PBLOCK + tid;
                int gx = 0, gy = 0, gz = 0;
                if (i < nsites) lmv[c] = link_mask(i, ownv[c], sv[c], gx, gy, gz);
                uint32_t mm = lmv[c];
                while (mm) {
                    const int b = __ffs(mm) - 1;
                    mm &= mm - 1;
                    z.add(b, gx, gy, gz, xc, nx, ny, nz);
                }
                const int cnt = __popc(lmv[c]);
                int incl = cnt;
                for (int o = 1; o < 64; o <<= 1) {
                    const int nb = __shfl_up(incl, o);
                    if (lane >= o) incl += nb;
                }
                offv[c] = incl - cnt;
                if (lane == 63) sh.wchunk[c][wv] = incl;
            }
        }
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int c = 0; c < P2B; ++c) {
            if (c < nch) {
                int before = 0, all = 0;
                for (int v = 0; v < PWAVES; ++v) {
                    const int t = sh.wchunk[c][v];
                    if (v < wv) before += t;
                    all += t;
                }
                offv[c] += total + before;
                total += all;
            }
        }
        if (total <= STAGE) {
#pragma unroll
            for (int c = 0; c < P2B; ++c) {
                uint32_t m2 = lmv[c];
                int idx = offv[c];
                while (m2) {
                    const int b = __ffs(m2) - 1;
                    m2 &= m2 - 1;
                    stage[idx++] = (uint32_t)sv[c] | ((uint32_t)b << SITE_BITS);
                }
            }
            __syncthreads();
            for (int j = tid; j < total; j += PBLOCK)
                if (j < lcap) L[j] = stage[j];
        } else {  // more links than the stage holds: each thread writes its own
#pragma unroll
            for (int c = 0; c < P2B; ++c) {
                uint32_t m2 = lmv[c];
                int idx = offv[c];
                while (m2) {
                    const int b = __ffs(m2) - 1;
                    m2 &= m2 - 1;
                    if (idx < lcap) L[idx] = (uint32_t)sv[c] | ((uint32_t)b << SITE_BITS);
                    ++idx;
                }
            }
        }
        running = total;
    } else {
        for (int base = 0; base < nsites; base += PBLOCK) {
            const int i = base + tid;
            uint32_t lm = 0;
            int s = 0, gx = 0, gy = 0, gz = 0;
            if (i < nsites && !((bits[i >> 5] >> (i & 31)) & 1u)) {
                int wx, wy;
                const int wz = divmod(divmod(i, wn[0], rw0, wx), wn[1], rw1, wy);
                const uint16_t own = om[wrap(lo[0] + wx, nx) + nx * (wrap(lo[1] + wy, ny) + ny * wrap(lo[2] + wz, nz))];
                lm = link_mask(i, own, s, gx, gy, gz);
            }
            const int cnt = __popc(lm);
            int incl = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int nb = __shfl_up(incl, o);
                if (lane >= o) incl += nb;
            }
            if (lane == 63) wtot[wv] = incl;
            __syncthreads();
            int off = incl - cnt, total = 0;
            for (int v = 0; v < PWAVES; ++v) {
                if (v < wv) off += wtot[v];
                total += wtot[v];
            }
            uint32_t mm = lm;
            while (mm) {
                const int b = __ffs(mm) - 1;
                mm &= mm - 1;
                z.add(b, gx, gy, gz, xc, nx, ny, nz);
            }
            for (int r0 = 0; r0 < total; r0 += STAGE) {
                uint32_t m2 = lm;
                int idx = off;
                while (m2) {
                    const int b = __ffs(m2) - 1;
                    m2 &= m2 - 1;
                    if (idx >= r0 && idx < r0 + STAGE) stage[idx - r0] = (uint32_t)s | ((uint32_t)b << SITE_BITS);
                    ++idx;
                }
                __syncthreads();
                const int n_r = min(STAGE, total - r0);
                for (int j = tid; j < n_r; j += PBLOCK) {
                    const int dst = running + r0 + j;
                    if (dst < lcap) L[dst] = stage[j];
                }
                __syncthreads();
            }
            running += total;
        }
    }
    if (running > lcap && tid == 0) atomicOr(a.flags, (int)F_LINKS);

    double all[15];
    for (int k = 0; k < 9; ++k) all[k] = z.zfw[k];
    for (int k = 0; k < 6; ++k) all[9 + k] = z.ztw[k];
    block_reduce<15>(all, red);
    const int iv[7] = {z.cnt6[0], z.cnt6[1], z.cnt6[2], z.cnt6[3], z.cnt6[4], z.cnt6[5], z.w36s};
    for (int k = 0; k < 7; ++k) {
        const int sm = wsumi(iv[k]);
        if (lane == 0) ired[k][wv] = sm;
    }
    __syncthreads();
    // one lane per output: the integer sums and the moments of the new link
    // set about this centre
    auto itot = [&](int k) {
        int t = 0;
        for (int v = 0; v < PWAVES; ++v) t += ired[k][v];
        return t;
    };
    if (tid == 36) {
        Pg->wsum = itot(6) / (double)WSCALE<Q>;
        Pg->nlinks = running < lcap ? running : lcap;
    } else if (tid >= 45 && tid < 69) {
        const int k = tid - 45;
        if (k < 6) Pg->zm0[k] = itot(k);
        else if (k < 15) Pg->zm1[k - 6] = red[k - 6][0];  // the block totals stay in LDS after the reduction
        else if (k < 21) Pg->zm2[k - 15] = red[9 + (k - 15)][0];
        else Pg->xref[k - 21] = P.xu[k - 21];
    }
}

// Steps 8-9 for particle p with its (new) state staged in LDS (P), in one
// work-group: scan, claims, links.  Only for a particle alone in its box
// (mode 0), or for adding / removing one particle at set-up (modes 1, 2),
// since the claims and the links here follow the scan without waiting for
// other work-groups.  stores_done: the bounce-back stores of the step are
// complete (a kernel boundary lies between); otherwise the claims wait for
// them first.
template <int ST, int Q>
__device__ __forceinline__ void remap_phase(const LaunchPart& a, int p, PartDev& P, RemapShm& sh, uint32_t* smem,
                                            bool stores_done) {
    uint32_t* bits = smem;
    uint32_t* stage = smem + a.lds_words;
    uint32_t* cand = stage;  // the candidate bits are consumed before the links are staged
    const BoxDesc& B = a.boxes[P.box];
    Win w;
    if (!window_of(a, P, B, w)) return;
    const int mode = a.mode;
    if (mode == 0 && !scan_needed(P)) {
        // no node can have changed side since the last scan
        if (a.near.flags) mark_near(a.near, B, w.lo, w.wn);
        return;
    }
    // an added particle stamps the cells it claims (with the set-up epoch),
    // so that only the particles whose window meets its nodes rebuild links
    const uint32_t ep = (mode == 1 && a.epoch) ? *a.epoch : 0u;
    double d0 = 0.0;
    // the band's list may take the whole of this kernel's LDS (bits, stage)
    // until a change needs the bits
    const int res = (mode == 0 && a.use_band && band_ok(P, d0))
                        ? band_pass<ST, Q>(a, p, P, B, w, bits, cand, smem, band_list_cap(a.lds_words), sh, 0u, d0)
                        : scan_pass<ST, Q>(a, p, P, B, w, bits, cand, sh, ep);
    if (mode == 2) {
        if (threadIdx.x == 0) a.parts[p].nlinks = 0;
        return;
    }
    if (mode == 0 && !(res & 1)) {
        // no node changed side: the link set and the link weights stay, no
        // mass or momentum moved
        if (a.near.flags) mark_near(a.near, B, w.lo, w.wn);
        return;
    }
    if (res & 2) {
        if (!stores_done) __syncthreads();  // the bounce-back writes before the covered-node reads
        claim_pass<ST, Q>(a, p, P, B, w, cand, sh);
    }
    link_pass<Q>(a, p, P, B, w, bits, stage, sh);
    if (mode == 0 && a.near.flags) mark_near(a.near, B, w.lo, w.wn);
}

template <int ST, int Q>
__global__ __launch_bounds__(PBLOCK) void k_particle_remap(LaunchPart a) {
    extern __shared__ uint32_t smem[];
    __shared__ PartDev P;
    __shared__ RemapShm sh;
    const int p = a.first + (int)blockIdx.x;
    stage_particle(a.parts + p, &P);
    remap_phase<ST, Q>(a, p, P, sh, smem, true);
}

// Steps 3-9 in one work-group, for boxes that hold one particle: the record
// is staged once, and the remap reads the bounce-back writes of its own
// work-group (no other particle writes this box).
template <int ST, int Q>
__global__ __launch_bounds__(PBLOCK) void k_particle_step(LaunchPart a) {
    extern __shared__ uint32_t smem[];
    __shared__ PartDev P;
    __shared__ union {
        SolveShm s;
        RemapShm r;
    } sh;
    const int p = a.first + (int)blockIdx.x;
    LinkRegs<typename Store<ST>::T> lr;
    load_particle<ST, Q>(a, p, &P, lr);
    solve_phase<ST, Q>(a, p, P, sh.s, lr, true);
    // the new state in LDS before the remap; the bounce-back stores may still
    // be in flight (the remap waits for them only before its claims)
    lds_barrier();
    remap_phase<ST, Q>(a, p, P, sh.r, smem, false);
}

// Boxes with several particles take three kernels per step, so that every
// particle's node-map update is complete before any particle claims a node,
// and every claim before any link list is rebuilt (the order of the paper's
// Appendix A: the whole node map at t+1, then links and drag matrices).
//
// 1. Steps 3-7 and pass 1 of the remap: releases, claim candidates (kept in
//    this particle's area of a.cand), stamps of the cells where owners change.
template <int ST, int Q>
__global__ __launch_bounds__(PBLOCK) void k_particle_solve_map(LaunchPart a) {
    extern __shared__ uint32_t smem[];  // the band's list
    __shared__ PartDev P;
    __shared__ union {
        SolveShm s;
        RemapShm r;
    } sh;
    const int p = a.first + (int)blockIdx.x;
    LinkRegs<typename Store<ST>::T> lr;
    load_particle<ST, Q>(a, p, &P, lr);
    solve_phase<ST, Q>(a, p, P, sh.s, lr, true);
    lds_barrier();
    PartDev* Pg = a.parts + p;
    const BoxDesc& B = a.boxes[P.box];
    Win w;
    int res = 0;
    if (window_of(a, P, B, w) && scan_needed(P)) {
        double d0 = 0.0;
        uint32_t* cand = a.cand + (size_t)p * a.lds_words;
        res = (a.use_band && band_ok(P, d0))
                  ? band_pass<ST, Q>(a, p, P, B, w, nullptr, cand, smem, band_list_cap(a.lds_words), sh.r, *a.epoch, d0)
                  : scan_pass<ST, Q>(a, p, P, B, w, nullptr, cand, sh.r, *a.epoch);
    }
    if (threadIdx.x == 0) {
        Pg->nchg = res & 1;
        Pg->ncand = (res >> 1) & 1;
    }
}

// 2. Claims of the candidates, after every particle's releases.
template <int ST, int Q>
__global__ __launch_bounds__(PBLOCK) void k_particle_claim(LaunchPart a) {
    __shared__ PartDev P;
    __shared__ RemapShm sh;
    const int p = a.first + (int)blockIdx.x;
    if (a.parts[p].ncand == 0) return;
    stage_particle(a.parts + p, &P);
    const BoxDesc& B = a.boxes[P.box];
    Win w;
    if (!window_of(a, P, B, w)) return;
    claim_pass<ST, Q>(a, p, P, B, w, a.cand + (size_t)p * a.lds_words, sh);
}

// 3. Links and their moments, from the complete node map, for a particle whose
//    own nodes changed or in whose window another particle's did (a cell of
//    the window carries this step's stamp).  With a.force_box >= 0 (after a
//    particle was added to that box at set-up, a.epoch then pointing at the
//    add's own epoch): the particles of that box whose window meets the
//    added particle's nodes.
// At most 128 VGPRs (four waves per SIMD): two work-groups per compute unit,
// so that the rebuilding work-groups of a large suspension are not queued
// behind one another (five values spill: six scratch stores and four
// reloads per thread, none in a loop).
template <int Q>
__global__ __launch_bounds__(PBLOCK, 4) void k_particle_links(LaunchPart a) {
    extern __shared__ uint32_t smem[];
    __shared__ PartDev P;
    __shared__ RemapShm sh;
    const int p = a.first + (int)blockIdx.x;
    if (a.force_box >= 0 && a.parts[p].box != a.force_box) return;
    stage_particle(a.parts + p, &P);
    const BoxDesc& B = a.boxes[P.box];
    Win w;
    if (!window_of(a, P, B, w)) return;
    const bool rebuild = (a.force_box < 0 && P.nchg != 0) || window_stamped(a, B, w, *a.epoch);
    if (rebuild) {
        uint32_t* bits = smem;
        bits_from_map(a, p, B, w, bits);
        link_pass<Q>(a, p, P, B, w, bits, smem + a.lds_words, sh);
    }
    if (a.force_box < 0 && a.near.flags) mark_near(a.near, B, w.lo, w.wn);
}

// Near set from the particles' current positions (set-up and re-tuning).
__global__ __launch_bounds__(256) void k_near_mark(LaunchPart a) {
    const PartDev& P = a.parts[a.first + blockIdx.x];
    const BoxDesc& B = a.boxes[P.box];
    int lo[3], wn[3];
    bool whole[3];
    particle_window(P, B, lo, wn, whole);
    mark_near(a.near, B, lo, wn);
}



// ------------------------------- launchers ----------------------------------

hipError_t launch_near_mark(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_near_mark, dim3(a.count), dim3(256), 0, st, a);
    return hipGetLastError();
}

// The bitmask of the window, and the link stage, which the candidate bits of
// the single-work-group remap share (they are consumed before links are
// staged).
size_t particle_remap_lds_bytes(int lds_words) {
    return (size_t)(lds_words + (lds_words > STAGE ? lds_words : STAGE)) * sizeof(uint32_t);
}

template <int ST, int Q>
struct SolveMapK {
    static void go(const LaunchPart& a, hipStream_t st) {
        hipLaunchKernelGGL((k_particle_solve_map<ST, Q>), dim3(a.count), dim3(PBLOCK),
                           particle_remap_lds_bytes(a.lds_words), st, a);
    }
};
template <int ST, int Q>
struct ClaimK {
    static void go(const LaunchPart& a, hipStream_t st) {
        hipLaunchKernelGGL((k_particle_claim<ST, Q>), dim3(a.count), dim3(PBLOCK), 0, st, a);
    }
};
template <template <int, int> class K, int Q>
static hipError_t by_storage(const LaunchPart& a, hipStream_t st) {
    switch (a.kp.storage) {
        case ST_F64: K<ST_F64, Q>::go(a, st); break;
        case ST_F32: K<ST_F32, Q>::go(a, st); break;
        case ST_F16: K<ST_F16, Q>::go(a, st); break;
        default: K<ST_BF16, Q>::go(a, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_particle_solve_map(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    return a.kp.q == 27 ? by_storage<SolveMapK, 27>(a, st) : by_storage<SolveMapK, 19>(a, st);
}

hipError_t launch_particle_claim(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    return a.kp.q == 27 ? by_storage<ClaimK, 27>(a, st) : by_storage<ClaimK, 19>(a, st);
}

hipError_t launch_particle_links(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    const size_t lds = particle_remap_lds_bytes(a.lds_words);
    if (a.kp.q == 27)
        hipLaunchKernelGGL((k_particle_links<27>), dim3(a.count), dim3(PBLOCK), lds, st, a);
    else
        hipLaunchKernelGGL((k_particle_links<19>), dim3(a.count), dim3(PBLOCK), lds, st, a);
    return hipGetLastError();
}

template <int ST, int Q>
static hipError_t remap_one(const LaunchPart& a, hipStream_t st) {
    const size_t lds = particle_remap_lds_bytes(a.lds_words);
    hipLaunchKernelGGL((k_particle_remap<ST, Q>), dim3(a.count), dim3(PBLOCK), lds, st, a);
    return hipGetLastError();
}

template <int Q>
static hipError_t step_q(const LaunchPart& a, hipStream_t st) {
    const size_t lds = particle_remap_lds_bytes(a.lds_words);
    switch (a.kp.storage) {
        case ST_F64: hipLaunchKernelGGL((k_particle_step<ST_F64, Q>), dim3(a.count), dim3(PBLOCK), lds, st, a); break;
        case ST_F32: hipLaunchKernelGGL((k_particle_step<ST_F32, Q>), dim3(a.count), dim3(PBLOCK), lds, st, a); break;
        case ST_F16: hipLaunchKernelGGL((k_particle_step<ST_F16, Q>), dim3(a.count), dim3(PBLOCK), lds, st, a); break;
        default: hipLaunchKernelGGL((k_particle_step<ST_BF16, Q>), dim3(a.count), dim3(PBLOCK), lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_particle_step(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    return a.kp.q == 27 ? step_q<27>(a, st) : step_q<19>(a, st);
}

template <int Q>
static hipError_t remap_q(const LaunchPart& a, hipStream_t st) {
    switch (a.kp.storage) {
        case ST_F64: return remap_one<ST_F64, Q>(a, st);
        case ST_F32: return remap_one<ST_F32, Q>(a, st);
        case ST_F16: return remap_one<ST_F16, Q>(a, st);
        default: return remap_one<ST_BF16, Q>(a, st);
    }
}

hipError_t launch_particle_remap(const LaunchPart& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    return a.kp.q == 27 ? remap_q<27>(a, st) : remap_q<19>(a, st);
}

}  // namespace lbd
