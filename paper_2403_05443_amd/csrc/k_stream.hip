// k_stream.hip - fused collide + stream over all boxes, plus the per-site
// initialisation and read-out kernels that see the lattice exactly as the
// collide kernel does.
//
// Storage: structure of arrays per box, f[dir * stride + site], in one of
// the conventions CV_PULL (ping-pong buffers: the value at (site, i) after a
// step is the post-collision population f*_i(site), the pre-collision
// population that site + c_i pulls at the next step, Sec. II.A:
// f_i(x + c_i, t + 1) = f*_i(x, t)) or CV_EVEN / CV_ODD (one buffer updated in
// place, alternating an even step that works on each node's own slots and an
// odd step that gathers from and scatters to the neighbours).  Link
// bounce-back on particles (Sec. II.B) writes the reflected value into the
// slot the fluid node reads next, so these kernels need no node map.  Moving
// walls (Sec. III.C set-up) are handled here: a population that would come
// out of a wall row is replaced by the node's own reflected population plus
// the moving-boundary term of eq. fb.
#include <hip/hip_ext.h>

#include <algorithm>

#include "lbell_dev.h"
#include "lbell_launch.h"

namespace lbd {

constexpr int XGROUP = 16;  // virtual blocks per XCD group of the grouped block order

template <int ST, int Q>
struct Pull {
    using S = Store<ST>;
    using T = typename S::T;
    using R = typename S::R;

    // Pre-collision populations of fluid site (x,y,z) as deviations, from
    // storage in convention CIN.
    // wsc: the scale of the result (1 for deviations; the storage scale when
    // inv_scale is 1 and the stored values are taken as they are)
    template <int CIN>
    static __device__ __forceinline__ void pull(const BoxDesc& B, const T* fi, int s,
                                                int x, int y, int z, R inv_scale, R rho0,
                                                bool walls, R (&f)[Q], R wsc = R(1)) {
#pragma clang fp contract(off)
        const int nx = B.nx, ny = B.ny, nz = B.nz;
        const long long st = B.stride;
        const int xs0 = x == nx - 1 ? 0 : x + 1, xs2 = x == 0 ? nx - 1 : x - 1;
        const int ys0 = y == ny - 1 ? 0 : y + 1, ys2 = y == 0 ? ny - 1 : y - 1;
        const int zs0 = z == nz - 1 ? 0 : z + 1, zs2 = z == 0 ? nz - 1 : z - 1;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            // source node x - c_i
            const int sx = cx(i) == 1 ? xs2 : (cx(i) == -1 ? xs0 : x);
            const int sy = cy(i) == 1 ? ys2 : (cy(i) == -1 ? ys0 : y);
            const int sz = cz(i) == 1 ? zs2 : (cz(i) == -1 ? zs0 : z);
            const int src = sx + nx * (sy + ny * sz);
            if (walls && cy(i) != 0 && (sy == 0 || sy == ny - 1)) {
                // f*_opp(i)(x) of the last step: its own opposite slot (pull),
                // its own slot i (even), the wall-row slot it was scattered to (odd)
                const double* uw = sy == 0 ? B.wall_lo : B.wall_hi;
                const R cu = (R)(cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2]);
                const long long off = CIN == CV_PULL ? (long long)opp(i) * st + s
                                    : (CIN == CV_EVEN ? (long long)i * st + s : (long long)opp(i) * st + src);
                f[i] = S::ld(fi + off, inv_scale) + (R)(6.0 * wgt<Q>(i)) * rho0 * cu * wsc;
            } else {
                const long long off = CIN == CV_PULL ? (long long)i * st + src
                                    : (CIN == CV_EVEN ? (long long)opp(i) * st + src : (long long)i * st + s);
                f[i] = S::ld(fi + off, inv_scale);
            }
        }
    }

    // The same in the convention held in a run-time value (read-out kernels).
    static __device__ __forceinline__ void pull_cv(int cv, const BoxDesc& B, const T* fi, int s, int x, int y,
                                                   int z, R inv_scale, R rho0, bool walls, R (&f)[Q]) {
        if (cv == CV_ODD) pull<CV_ODD>(B, fi, s, x, y, z, inv_scale, rho0, walls, f);
        else if (cv == CV_EVEN) pull<CV_EVEN>(B, fi, s, x, y, z, inv_scale, rho0, walls, f);
        else pull<CV_PULL>(B, fi, s, x, y, z, inv_scale, rho0, walls, f);
    }
};

// c_i . v with the zero components of c_i left out and the unit ones taken
// as a sign: under IEEE rules 0 * v (v might be infinite) and 1 * v are not
// folded away by the compiler, and they were most of the collision's
// instructions.  The value equals the plain dot product (up to the sign of a
// zero result).  i is a compile-time constant after unrolling, so every
// branch here folds.
template <typename R>
__device__ __forceinline__ R dotc(int i, R vx, R vy, R vz) {
    R s = R(0);
    bool any = false;
    if (cx(i) != 0) {
        s = cx(i) > 0 ? vx : -vx;
        any = true;
    }
    if (cy(i) != 0) {
        const R t = cy(i) > 0 ? vy : -vy;
        s = any ? s + t : t;
        any = true;
    }
    if (cz(i) != 0) {
        const R t = cz(i) > 0 ? vz : -vz;
        s = any ? s + t : t;
    }
    return s;
}

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// 1 / x: the hardware reciprocal in FP32 (1 ulp; every variant uses it), the
// correctly rounded quotient in FP64
__device__ __forceinline__ float rcpr(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpr(double x) { return 1.0 / x; }

// Collision on deviations d_i = f_i - w_i rho0 (algebraically identical to
// the full-population forms of Sec. II.A).  FP contraction is off and the
// fused multiply-adds are written out: every collide-stream variant then
// rounds identically, so results never depend on which variant the tuner
// picked.
// SCALED (the half formats): f holds the stored, scaled deviations
// sc (f_i - w_i rho0) and the result is scaled the same way, so that loads
// and stores need no multiply per population; the density and velocity are
// formed unscaled (isc = 1 / sc), and w rho and the counter-force term carry
// the scale.  sc is a power of two, so every product and sum here is the
// unscaled one times sc exactly: the results are those of scaling at the
// loads and stores, bit for bit.  The regularised collision unscales and
// rescales instead.
template <typename R, int COLL, int Q, bool SCALED = false>
__device__ __forceinline__ void collide(R (&f)[Q], R rho0, R om, R omm, bool cf, R g0, R g1, R g2, R sc = R(1),
                                        R isc = R(1)) {
#pragma clang fp contract(off)
    if constexpr (SCALED && COLL == 2) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] *= isc;
        collide<R, COLL, Q, false>(f, rho0, om, omm, cf, g0, g1, g2);
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] *= sc;
        return;
    }
    R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += f[i];
        if (cx(i)) jx += cx(i) * f[i];
        if (cy(i)) jy += cy(i) * f[i];
        if (cz(i)) jz += cz(i) * f[i];
    }
    // drho, j are scaled like f when SCALED; rho and u are not
    const R rho = SCALED ? rho0 + drho * isc : rho0 + drho;
    const R ir = SCALED ? isc * rcpr(rho) : rcpr(rho);
    const R ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const R rs = SCALED ? rho * sc : rho;  // w rs: the scaled w rho
    const R usq = R(1.5) * fmar(ux, ux, fmar(uy, uy, uz * uz));
    // w rho and w drho per weight class (the rest, the axes, the edges, the
    // corners); i is a compile-time constant after unrolling
    auto wcls = [](int i) { return i == 0 ? 0 : (i <= 6 ? 1 : (i <= 18 ? 2 : 3)); };
    R wr[4], wd[4], w3r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int rep = k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? 7 : 19));
        wr[k] = R(wgt<Q>(rep)) * rs;
        wd[k] = R(wgt<Q>(rep)) * drho;
        w3r[k] = R(3) * wr[k];
    }
    if (COLL == 0) {  // BGK: f_eq = w (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2))
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R cu = dotc<R>(i, ux, uy, uz);
            const R feq = fmar(wr[wcls(i)], fmar(cu, fmar(R(4.5), cu, R(3)), -usq), wd[wcls(i)]);
            f[i] = fmar(-om, f[i] - feq, f[i]);
        }
    } else if (COLL == 1) {  // TRT
        f[0] = fmar(-om, f[0] - fmar(-wr[0], usq, wd[0]), f[0]);
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            // symmetric and antisymmetric parts of the pair (i, opp(i)) and
            // of its equilibrium: e+ = w (drho + rho (4.5 cu^2 - 1.5 u^2)),
            // e- = 3 w rho cu; a = om+ (f+ - e+), b = om- (f- - e-)
            const int o = i + 1, k = wcls(i);
            const R cu = dotc<R>(i, ux, uy, uz);
            const R ep = fmar(wr[k], fmar(R(4.5) * cu, cu, -usq), wd[k]);
            const R em = w3r[k] * cu;
            const R s = f[i] + f[o], d = f[i] - f[o];
            const R a = fmar(R(0.5) * om, s, -(om * ep));
            const R b = fmar(R(0.5) * omm, d, -(omm * em));
            f[i] = f[i] - (a + b);
            f[o] = f[o] - (a - b);
        }
    } else {  // hydrodynamic modes relaxed with tau, ghost modes to equilibrium
        R pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (cx(i)) pxx += f[i];
            if (cy(i)) pyy += f[i];
            if (cz(i)) pzz += f[i];
            if (cx(i) && cy(i)) pxy += R(cx(i) * cy(i)) * f[i];
            if (cx(i) && cz(i)) pxz += R(cx(i) * cz(i)) * f[i];
            if (cy(i) && cz(i)) pyz += R(cy(i) * cz(i)) * f[i];
        }
        // X = rho u u + (1 - 1/tau) (sum d c c - drho/3 I - rho u u)
        const R k1 = R(1) - om, d3 = drho * R(1.0 / 3.0);
        const R xxx = rho * ux * ux + k1 * (pxx - d3 - rho * ux * ux);
        const R xyy = rho * uy * uy + k1 * (pyy - d3 - rho * uy * uy);
        const R xzz = rho * uz * uz + k1 * (pzz - d3 - rho * uz * uz);
        const R xxy = rho * ux * uy + k1 * (pxy - rho * ux * uy);
        const R xxz = rho * ux * uz + k1 * (pxz - rho * ux * uz);
        const R xyz = rho * uy * uz + k1 * (pyz - rho * uy * uz);
        const R tr3 = (xxx + xyy + xzz) * R(1.0 / 3.0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R cu = dotc<R>(i, ux, uy, uz);
            R cxc = 0;
            if (cx(i)) cxc += xxx;
            if (cy(i)) cxc += xyy;
            if (cz(i)) cxc += xzz;
            if (cx(i) && cy(i)) cxc += R(2 * cx(i) * cy(i)) * xxy;
            if (cx(i) && cz(i)) cxc += R(2 * cx(i) * cz(i)) * xxz;
            if (cy(i) && cz(i)) cxc += R(2 * cy(i) * cz(i)) * xyz;
            f[i] = R(wgt<Q>(i)) * (drho + R(3) * rho * cu + R(4.5) * (cxc - tr3));
        }
    }
    if (cf) {  // uniform counter-force, w_i (c_i . g) / c_s^2 (opposite for opp(i))
        const R r0 = SCALED ? rho0 * sc : rho0;
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const R t = R(3.0 * wgt<Q>(i)) * r0 * dotc<R>(i, g0, g1, g2);
            f[i] += t;
            f[i + 1] -= t;
        }
    }
}

// One site of the generic tile kernel: read the pre-collision populations
// (convention CIN), collide, store the post-collision ones (convention COUT).
template <int ST, int COLL, bool WALLS, bool NT, int CIN, int COUT, int Q>
__device__ __forceinline__ void site_update(const BoxDesc* __restrict__ boxes, const int* __restrict__ tile_box,
                                            const typename Store<ST>::T* fin, typename Store<ST>::T* fout,
                                            const KParams& kp, int tile, uint32_t step) {
    using S = Store<ST>;
    using R = typename S::R;
    const int bi = tile_box[tile];
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    const int nx = B.nx, ny = B.ny;
    int x, y;
    const int z = div_magic(div_magic(s, nx, B.mnx, B.lnx, x), ny, B.mny, B.lny, y);
    const bool walls = WALLS && B.walls;
    if (walls && (y == 0 || y == ny - 1)) return;
    // the half formats collide on the scaled values as stored (see collide)
    constexpr bool SC = ST >= ST_F16;
    const R inv = (R)kp.inv_scale, scl = (R)kp.scale, rho0 = (R)kp.rho0;
    R f[Q];
    Pull<ST, Q>::template pull<CIN>(B, fin + B.foff, s, x, y, z, SC ? R(1) : inv, rho0, walls, f, SC ? scl : R(1));
    R g0 = 0, g1 = 0, g2 = 0;
    const bool cf = B.counterforce != 0;
    if (cf) {  // uniform force density on all matter of the box (fluid and particles)
        g0 = (R)B.gcf[0];
        g1 = (R)B.gcf[1];
        g2 = (R)B.gcf[2];
    }
    collide<R, COLL, Q, SC>(f, rho0, (R)kp.omega, (R)kp.omega_m, cf, g0, g1, g2, scl, inv);
    typename S::T* fo = fout + B.foff;
    // the dither is a function of (node, direction, step) in every convention
    const uint32_t seed = ST >= ST_F16 ? dither_seed((uint32_t)s, step) : 0u;
    const int nz = B.nz;
    const int xp = x == nx - 1 ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
    const int yp = y == ny - 1 ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
    const int zp = z == nz - 1 ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t r = ST >= ST_F16 ? dither_bits(seed, i) : 0u;
        long long off;
        if (COUT == CV_ODD) {  // scattered to the node it streams to
            const int dx = cx(i) == 1 ? xp : (cx(i) == -1 ? xm : x);
            const int dy = cy(i) == 1 ? yp : (cy(i) == -1 ? ym : y);
            const int dz = cz(i) == 1 ? zp : (cz(i) == -1 ? zm : z);
            off = (long long)i * B.stride + (dx + nx * (dy + ny * dz));
        } else {
            off = (long long)(COUT == CV_EVEN ? opp(i) : i) * B.stride + s;
        }
        if constexpr (NT) {
            typename S::T v;
            S::st_dither(&v, f[i], SC ? R(1) : scl, r);
            __builtin_nontemporal_store(v, fo + off);
        } else {
            S::st_dither(fo + off, f[i], SC ? R(1) : scl, r);
        }
    }
}

// Generic tile kernel over every box of the context.  A virtual block covers
// SPT consecutive 256-site tiles (one site per thread and tile).  Block order
// (the hardware deals consecutive blocks out to the 8 XCDs in turn, and
// neighbouring tiles share cache lines at their edges, which one XCD's L2
// serves once): XCD = 1, the grid is 8 * m blocks and the virtual blocks are
// cut into 8 contiguous ranges, range k walked by the blocks with
// blockIdx % 8 == k (a grid smaller than the work, a persistent launch, walks
// its range in strides of m); XCD = 2, the blocks of XCD k take groups of
// XGROUP consecutive virtual blocks, and the groups of the 8 XCDs alternate,
// so the sweep keeps the plain order at the scale of 8 XGROUP blocks while
// most tile edges stay within one L2.  XCD = 0: block b takes virtual blocks
// b, b + grid, ...  NT: stores that
// do not allocate in the caches.  The near-set parts (part 1, 2) use SPT = 1
// and the plain order only.
template <int ST, int COLL, bool WALLS, int SPT, int XCD, bool NT, int Q>
__global__ __launch_bounds__(TILE) void k_collide_stream(const BoxDesc* __restrict__ boxes,
                                                         const BoxRT* __restrict__ rt,
                                                         const int* __restrict__ tile_box,
                                                         const typename Store<ST>::T* __restrict__ fin,
                                                         typename Store<ST>::T* __restrict__ fout,
                                                         KParams kp, int part, const uint32_t* __restrict__ nflags,
                                                         const int* __restrict__ nlist,
                                                         const int* __restrict__ ncount, uint32_t epoch,
                                                         int* __restrict__ next_count, int ntiles,
                                                         const uint32_t* __restrict__ step_in,
                                                         uint32_t* __restrict__ step_out) {
    const uint32_t step = *step_in;  // the step being computed (read by every block)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (next_count) *next_count = 0;
        *step_out = step + 1;  // the other parity's slot, read by the next step
    }
    if (SPT == 1 && XCD == 0 && part != 0) {
        int tile = blockIdx.x;
        if (part == 2) {
            if (tile >= *ncount) return;
            tile = nlist[tile];
        } else if (nflags[tile] == epoch) {
            return;
        }
        site_update<ST, COLL, WALLS, NT, CV_PULL, CV_PULL, Q>(boxes, tile_box, fin, fout, kp, tile, step);
        return;
    }
    const int nvb = (ntiles + SPT - 1) / SPT;
    int v, vend, vstep;
    if (XCD == 1) {
        const int m = (int)gridDim.x >> 3, chunk = (nvb + 7) >> 3, k = (int)(blockIdx.x & 7);
        v = k * chunk + (int)(blockIdx.x >> 3);
        vend = min(nvb, (k + 1) * chunk);
        vstep = m;
    } else if (XCD == 2) {
        // walks this XCD's local index J; v(J) = groups of XGROUP, XCDs interleaved
        v = (int)(blockIdx.x >> 3);
        vend = ((nvb + 8 * XGROUP - 1) / (8 * XGROUP)) * XGROUP;
        vstep = (int)gridDim.x >> 3;
    } else {
        v = blockIdx.x;
        vend = nvb;
        vstep = gridDim.x;
    }
    for (; v < vend; v += vstep) {
        const int vb = XCD == 2 ? (v / XGROUP) * (8 * XGROUP) + (int)(blockIdx.x & 7) * XGROUP + v % XGROUP : v;
        if (XCD == 2 && vb >= nvb) continue;
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int tile = vb * SPT + k;
            if (tile < ntiles) site_update<ST, COLL, WALLS, NT, CV_PULL, CV_PULL, Q>(boxes, tile_box, fin, fout, kp, tile, step);
        }
    }
}

// In-place step over one buffer: CIN = CV_ODD runs the even step (each node
// reads and rewrites its own slots), CIN = CV_EVEN the odd step (gather from
// and scatter to the neighbours).  Every slot is read and written by one
// thread only, so no block depends on another.  Block order as the generic
// kernel's; wall rows are not updated.
template <int ST, int COLL, bool WALLS, int SPT, int XCD, bool NT, int CIN, int Q>
__global__ __launch_bounds__(TILE) void k_collide_stream_aa(const BoxDesc* __restrict__ boxes,
                                                            const int* __restrict__ tile_box,
                                                            typename Store<ST>::T* __restrict__ f, KParams kp,
                                                            int ntiles, const uint32_t* __restrict__ step_in,
                                                            uint32_t* __restrict__ step_out) {
    constexpr int COUT = CIN == CV_ODD ? CV_EVEN : CV_ODD;
    const uint32_t step = *step_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) *step_out = step + 1;
    const int nvb = (ntiles + SPT - 1) / SPT;
    int v, vend, vstep;
    if (XCD == 1) {
        const int m = (int)gridDim.x >> 3, chunk = (nvb + 7) >> 3, k = (int)(blockIdx.x & 7);
        v = k * chunk + (int)(blockIdx.x >> 3);
        vend = min(nvb, (k + 1) * chunk);
        vstep = m;
    } else if (XCD == 2) {
        // walks this XCD's local index J; v(J) = groups of XGROUP, XCDs interleaved
        v = (int)(blockIdx.x >> 3);
        vend = ((nvb + 8 * XGROUP - 1) / (8 * XGROUP)) * XGROUP;
        vstep = (int)gridDim.x >> 3;
    } else {
        v = blockIdx.x;
        vend = nvb;
        vstep = gridDim.x;
    }
    for (; v < vend; v += vstep) {
        const int vb = XCD == 2 ? (v / XGROUP) * (8 * XGROUP) + (int)(blockIdx.x & 7) * XGROUP + v % XGROUP : v;
        if (XCD == 2 && vb >= nvb) continue;
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int tile = vb * SPT + k;
            if (tile < ntiles) site_update<ST, COLL, WALLS, NT, CIN, COUT, Q>(boxes, tile_box, f, f, kp, tile, step);
        }
    }
}

// Moves every population from its slot in convention cs (buffer src) to its
// slot in convention cd (buffer dst), wall and particle nodes included: a
// permutation of the slots (post_slot is one-to-one per direction), exact.
template <typename T>
__global__ __launch_bounds__(TILE) void k_relayout(const BoxDesc* __restrict__ boxes, const int* __restrict__ tile_box,
                                                   const T* __restrict__ src, T* __restrict__ dst, int cs, int cd,
                                                   int q) {
    const int tile = blockIdx.x;
    const BoxDesc& B = boxes[tile_box[tile]];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
#pragma unroll
    for (int i = 0; i < q; ++i) {
        int ds, ss, dd, sd;
        post_slot(cs, i, x, y, z, nx, ny, nz, ds, ss);
        post_slot(cd, i, x, y, z, nx, ny, nz, dd, sd);
        dst[B.foff + (long long)dd * B.stride + sd] = src[B.foff + (long long)ds * B.stride + ss];
    }
}

// Row-wave variant for boxes with nx = 64 K: one wavefront owns one x-row,
// lane l holds the K consecutive sites [K l, K l + K).  Every direction plane
// is read with one aligned K-wide vector load per lane; the +-1 shift of the
// directions with c_x != 0 moves one element across lanes with a wave
// rotation (ds_bpermute), which is also the periodic wrap of the row.
template <typename T, int K>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(K)));
};
template <typename T>
struct VecOf<T, 1> {
    typedef T type;
};

template <typename T, typename R, int K, int ST>
__device__ __forceinline__ void ld_vec(const T* p, R inv, R (&v)[K]) {
    using V = typename VecOf<T, K>::type;
    const V x = *reinterpret_cast<const V*>(p);
    if constexpr (K == 1) {
        v[0] = Store<ST>::ld(&x, inv);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T e = x[j];
            v[j] = Store<ST>::ld(&e, inv);
        }
    }
}

// K consecutive sites (dither seeds seed[j]) of direction dir; half formats
// round with the same dither as the generic kernel
template <typename T, typename R, int K, int ST, bool NT>
__device__ __forceinline__ void st_vec(T* p, R scl, const R (&v)[K], const uint32_t (&seed)[K], int dir) {
    using V = typename VecOf<T, K>::type;
    V x;
    if constexpr (K == 1) {
        Store<ST>::st_dither(&x, v[0], scl, ST >= ST_F16 ? dither_bits(seed[0], dir) : 0u);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            T e;
            Store<ST>::st_dither(&e, v[j], scl, ST >= ST_F16 ? dither_bits(seed[j], dir) : 0u);
            x[j] = e;
        }
    }
    if constexpr (NT)
        __builtin_nontemporal_store(x, reinterpret_cast<V*>(p));
    else
        *reinterpret_cast<V*>(p) = x;
}

template <int ST, int COLL, bool WALLS, int K, bool NT, int Q>
__global__ __launch_bounds__(256) void k_collide_stream_rows(const BoxDesc* __restrict__ boxes,
                                                             const BoxRT* __restrict__ rt, int bi,
                                                             const typename Store<ST>::T* __restrict__ fin,
                                                             typename Store<ST>::T* __restrict__ fout,
                                                             KParams kp, int part,
                                                             const uint32_t* __restrict__ nflags,
                                                             const int* __restrict__ nlist,
                                                             const int* __restrict__ ncount, uint32_t epoch,
                                                             int* __restrict__ next_count,
                                                             const uint32_t* __restrict__ step_in,
                                                             uint32_t* __restrict__ step_out) {
#pragma clang fp contract(off)
    using S = Store<ST>;
    using T = typename S::T;
    using R = typename S::R;
    const uint32_t step = *step_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (next_count) *next_count = 0;
        *step_out = step + 1;
    }
    const BoxDesc& B = boxes[bi];
    const int ny = B.ny, nz = B.nz, nx = 64 * K;
    const int lane = threadIdx.x & 63;
    int rb = blockIdx.x;
    if (part == 2) {
        if (rb >= *ncount) return;
        rb = nlist[rb];
    } else if (part == 1 && nflags[rb] == epoch) {
        return;
    }
    const int row = rb * 4 + (threadIdx.x >> 6);
    if (row >= ny * nz) return;
    const int y = row % ny, z = row / ny;
    const bool walls = WALLS && B.walls;
    if (walls && (y == 0 || y == ny - 1)) return;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    const long long st = B.stride;
    const T* fi = fin + B.foff;
    const int x0 = K * lane;
    // the half formats collide on the scaled values as stored (see collide)
    constexpr bool SC = ST >= ST_F16;
    const R inv = (R)kp.inv_scale, scl = (R)kp.scale, rho0 = (R)kp.rho0;
    const R ldi = SC ? R(1) : inv, sts = SC ? R(1) : scl, wsc = SC ? scl : R(1);
    const int up = (lane + 63) & 63, dn = (lane + 1) & 63;
    R f[K][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int sy = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
        const int sz = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
        R v[K];
        if (walls && cy(i) != 0 && (sy == 0 || sy == ny - 1)) {
            const double* uw = sy == 0 ? B.wall_lo : B.wall_hi;
            const R cu = (R)(cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2]);
            ld_vec<T, R, K, ST>(fi + (long long)opp(i) * st + (long long)nx * (y + ny * z) + x0, ldi, v);
#pragma unroll
            for (int j = 0; j < K; ++j) f[j][i] = v[j] + (R)(6.0 * wgt<Q>(i)) * rho0 * cu * wsc;
            continue;
        }
        ld_vec<T, R, K, ST>(fi + (long long)i * st + (long long)nx * (sy + ny * sz) + x0, ldi, v);
        if (cx(i) == 1) {  // source x - 1
            const R carry = __shfl(v[K - 1], up);
#pragma unroll
            for (int j = K - 1; j > 0; --j) v[j] = v[j - 1];
            v[0] = carry;
        } else if (cx(i) == -1) {  // source x + 1
            const R carry = __shfl(v[0], dn);
#pragma unroll
            for (int j = 0; j < K - 1; ++j) v[j] = v[j + 1];
            v[K - 1] = carry;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) f[j][i] = v[j];
    }
    R g0 = 0, g1 = 0, g2 = 0;
    const bool cf = B.counterforce != 0;
    if (cf) {  // uniform force density on all matter of the box (fluid and particles)
        g0 = (R)B.gcf[0];
        g1 = (R)B.gcf[1];
        g2 = (R)B.gcf[2];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) collide<R, COLL, Q, SC>(f[j], rho0, (R)kp.omega, (R)kp.omega_m, cf, g0, g1, g2, scl, inv);
    T* fo = fout + B.foff + (long long)nx * (y + ny * z) + x0;
    uint32_t seed[K];
#pragma unroll
    for (int j = 0; j < K; ++j) seed[j] = ST >= ST_F16 ? dither_seed((uint32_t)(nx * (y + ny * z) + x0 + j), step) : 0u;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = f[j][i];
        st_vec<T, R, K, ST, NT>(fo + (long long)i * st, sts, v, seed, i);
    }
}

// Initial state: every slot holds the pre-collision population its reader
// pulls at the first step, f_eq(rho0, u0) plus the first-order
// non-equilibrium part of the Couette profile (zero at rest).
template <int ST, int Q>
__global__ __launch_bounds__(TILE) void k_init(const BoxDesc* __restrict__ boxes,
                                               const int* __restrict__ tile_box,
                                               typename Store<ST>::T* __restrict__ f0,
                                               typename Store<ST>::T* __restrict__ f1,
                                               const int* __restrict__ box_init, KParams kp) {
    using S = Store<ST>;
    const int tile = blockIdx.x;
    const int bi = tile_box[tile];
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
    const bool couette = box_init[bi] == 1 && B.walls;
    const double H = ny - 2.0;
    double gr[3] = {0, 0, 0};
    if (couette)
        for (int k = 0; k < 3; ++k) gr[k] = (B.wall_hi[k] - B.wall_lo[k]) / H;
    const double tau = 1.0 / kp.omega, rho0 = kp.rho0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // reader of slot (s, i) is node s + c_i
        int yd = y + cy(i);
        double val = 0.0;
        const bool wall_here = B.walls && (y == 0 || y == ny - 1);
        auto dev = [&](int j, int yy) {  // pre-collision deviation of f_j at fluid row yy
            if (!couette) return 0.0;
            double u[3];
            for (int k = 0; k < 3; ++k) u[k] = B.wall_lo[k] + gr[k] * (yy - 0.5);
            const double cu = cx(j) * u[0] + cy(j) * u[1] + cz(j) * u[2];
            const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            const double qg = cy(j) * (cx(j) * gr[0] + cz(j) * gr[2]);
            return wgt<Q>(j) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu) - tau * wgt<Q>(j) * rho0 * 3.0 * qg;
        };
        if (!wall_here) {
            if (B.walls && (yd == 0 || yd == ny - 1)) {
                // slot consumed by bounce-back at s: f_opp(i)(s) = slot + 6 w (u_w . c_opp(i))
                const int o = opp(i);
                const double* uw = yd == 0 ? B.wall_lo : B.wall_hi;
                const double cu = cx(o) * uw[0] + cy(o) * uw[1] + cz(o) * uw[2];
                val = dev(o, y) - 6.0 * wgt<Q>(o) * rho0 * cu;
            } else {
                val = dev(i, wrap(yd, ny));
            }
        }
        (void)nz;
        (void)x;
        (void)z;
        S::st64(f0 + B.foff + (long long)i * B.stride + s, val, kp.scale);
        S::st64(f1 + B.foff + (long long)i * B.stride + s, val, kp.scale);
    }
}

// Pre-collision density / velocity of fluid sites of one box, for a chunk of
// sites [s0, s0 + count): out[4*k] = rho, out[4*k+1..3] = u (zeros elsewhere).
template <int ST, int Q>
__global__ __launch_bounds__(TILE) void k_fields(const BoxDesc* __restrict__ boxes, int bi,
                                                 const uint16_t* __restrict__ omap,
                                                 const typename Store<ST>::T* __restrict__ fin,
                                                 int s0, int count, double* __restrict__ out,
                                                 KParams kp) {
    using R = typename Store<ST>::R;
    const BoxDesc& B = boxes[bi];
    const int k = blockIdx.x * TILE + (int)threadIdx.x;
    if (k >= count) return;
    const int s = s0 + k;
    double rho = 0, u[3] = {0, 0, 0};
    if (omap[B.ooff + s] == 0) {
        const int nx = B.nx, ny = B.ny;
        const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
        R f[Q];
        Pull<ST, Q>::pull_cv(kp.conv, B, fin + B.foff, s, x, y, z, (R)kp.inv_scale, (R)kp.rho0, B.walls != 0, f);
        double d = 0, j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            d += (double)f[i];
            j[0] += cx(i) * (double)f[i];
            j[1] += cy(i) * (double)f[i];
            j[2] += cz(i) * (double)f[i];
        }
        rho = kp.rho0 + d;
        for (int c = 0; c < 3; ++c) u[c] = j[c] / rho;
    }
    out[4 * k] = rho;
    out[4 * k + 1] = u[0];
    out[4 * k + 2] = u[1];
    out[4 * k + 3] = u[2];
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-block sums over fluid sites: [count, sum(d rho), j_x, j_y, j_z, non-finite].
template <int ST, int Q>
__global__ __launch_bounds__(TILE) void k_moments(const BoxDesc* __restrict__ boxes, int bi,
                                                  const uint16_t* __restrict__ omap,
                                                  const typename Store<ST>::T* __restrict__ fin,
                                                  double* __restrict__ partial, KParams kp) {
    using R = typename Store<ST>::R;
    const BoxDesc& B = boxes[bi];
    const int s = blockIdx.x * TILE + (int)threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (s < B.n && omap[B.ooff + s] == 0) {
        const int nx = B.nx, ny = B.ny;
        const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
        R f[Q];
        Pull<ST, Q>::pull_cv(kp.conv, B, fin + B.foff, s, x, y, z, (R)kp.inv_scale, (R)kp.rho0, B.walls != 0, f);
        v[0] = 1.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double fi = (double)f[i];
            if (!isfinite(fi)) v[5] += 1.0;
            v[1] += fi;
            v[2] += cx(i) * fi;
            v[3] += cy(i) * fi;
            v[4] += cz(i) * fi;
        }
    }
    __shared__ double red[6][TILE / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 6; ++k) {
        const double w = wave_sum_d(v[k]);
        if (lane == 0) red[k][wv] = w;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double a = 0;
        for (int w = 0; w < TILE / 64; ++w) a += red[threadIdx.x][w];
        partial[(long long)blockIdx.x * 6 + threadIdx.x] = a;
    }
}

// Flow energy per tile for the warm-start monitor: the sum over the tile's
// fluid sites of |j|^2, j = sum_i (f_i - w_i rho0) c_i the momentum density,
// for boxes whose monitor is pending (0 elsewhere).
template <int ST, int Q>
__global__ __launch_bounds__(TILE) void k_box_energy(const BoxDesc* __restrict__ boxes,
                                                     const int* __restrict__ tile_box,
                                                     const uint16_t* __restrict__ omap,
                                                     const typename Store<ST>::T* __restrict__ fin,
                                                     const BoxMon* __restrict__ mon, double* __restrict__ partial,
                                                     KParams kp) {
    using R = typename Store<ST>::R;
    const int tile = blockIdx.x;
    const int bi = tile_box[tile];
    if (mon[bi].status != MON_PENDING) {  // uniform over the block
        if (threadIdx.x == 0) partial[tile] = 0.0;
        return;
    }
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    double e = 0.0;
    if (s < B.n && omap[B.ooff + s] == 0) {
        const int nx = B.nx, ny = B.ny;
        const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
        R f[Q];
        Pull<ST, Q>::pull_cv(kp.conv, B, fin + B.foff, s, x, y, z, (R)kp.inv_scale, (R)kp.rho0, B.walls != 0, f);
        double j[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            j[0] += cx(i) * (double)f[i];
            j[1] += cy(i) * (double)f[i];
            j[2] += cz(i) * (double)f[i];
        }
        e = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    }
    __shared__ double red[TILE / 64];
    const double w = wave_sum_d(e);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int k = 0; k < TILE / 64; ++k) a += red[k];
        partial[tile] = a;
    }
}

template <int ST>
__global__ void k_poke(const BoxDesc* __restrict__ boxes, int bi, typename Store<ST>::T* __restrict__ f,
                       int s, int dir, double val, KParams kp) {
    const BoxDesc& B = boxes[bi];
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
    int d, slot;
    pre_slot_open(kp.conv, dir, x, y, z, nx, ny, nz, d, slot);
    Store<ST>::st64(f + B.foff + (long long)d * B.stride + slot, val, kp.scale);
}

// Plain device copy with 16-byte accesses, four per thread per iteration:
// the achievable read+write bandwidth reference for the roofline, and the
// known-size kernel that calibrates the HBM byte counters.
__global__ __launch_bounds__(256) void k_copy_probe(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                    size_t n16) {
    // one 16-byte element per thread over a grid that covers the buffer: the
    // fastest of the copy shapes measured (grid-stride loops with 1-8 elements
    // per thread on 4-32 blocks per CU reach 4.1-5.7 TB/s, this 6.2 TB/s)
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, bytes / 16);
    return hipGetLastError();
}

// ------------------------------- launchers ----------------------------------

// A collide-stream launch; with timing events in the arguments they receive
// the kernel's own start and end (no stream work between them).
#define K1_LAUNCH(KERNEL, G, B, ST, ...)                                                   \
    do {                                                                                 \
        if (a.ev_start)                                                                  \
            hipExtLaunchKernelGGL(KERNEL, G, B, 0, ST, a.ev_start, a.ev_stop, 0, __VA_ARGS__); \
        else                                                                             \
            hipLaunchKernelGGL(KERNEL, G, B, 0, ST, __VA_ARGS__);                          \
    } while (0)

template <int ST, int COLL, bool WALLS, int SPT, int XCD, bool NT, int Q>
static hipError_t cs_one(const LaunchCS& a, hipStream_t st) {
    using T = typename Store<ST>::T;
    const int nvb = (a.ntiles + SPT - 1) / SPT;
    int g;
    if (a.part == 2) g = a.near_grid;
    else if (XCD) g = 8 * (a.grid > 0 ? std::max(1, a.grid / 8) : (nvb + 7) / 8);
    else g = a.grid > 0 ? std::min(a.grid, nvb) : nvb;
    if (g == 0 || a.ntiles == 0) return hipSuccess;
    K1_LAUNCH((k_collide_stream<ST, COLL, WALLS, SPT, XCD, NT, Q>), dim3(g), dim3(TILE), st, a.boxes, a.rt,
              a.tile_box, (const T*)a.fin, (T*)a.fout, a.kp, a.part, a.near_flags, a.near_list, a.near_count,
              a.near_epoch, a.next_count, a.ntiles, a.step_in, a.step_out);
    return hipGetLastError();
}

template <int ST, int COLL, bool WALLS, int SPT, int XCD, bool NT, int Q>
static hipError_t aa_one(const LaunchCS& a, hipStream_t st) {
    using T = typename Store<ST>::T;
    const int nvb = (a.ntiles + SPT - 1) / SPT;
    const int g = XCD ? 8 * ((nvb + 7) / 8) : nvb;
    if (a.ntiles == 0) return hipSuccess;
    if (a.kp.conv == CV_ODD)
        K1_LAUNCH((k_collide_stream_aa<ST, COLL, WALLS, SPT, XCD, NT, CV_ODD, Q>), dim3(g), dim3(TILE), st, a.boxes,
                  a.tile_box, (T*)a.fout, a.kp, a.ntiles, a.step_in, a.step_out);
    else if (a.kp.conv == CV_EVEN)
        K1_LAUNCH((k_collide_stream_aa<ST, COLL, WALLS, SPT, XCD, NT, CV_EVEN, Q>), dim3(g), dim3(TILE), st, a.boxes,
                  a.tile_box, (T*)a.fout, a.kp, a.ntiles, a.step_in, a.step_out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// D3Q27 takes the one-tile-per-block shapes only (plain or XCD-chunked, pull
// or in place); the tuner offers no other.
template <int ST, int COLL, bool WALLS, int Q>
static hipError_t cs_shape(const LaunchCS& a, hipStream_t st) {
    const int key = a.spt * 8 + a.xcd * 2 + (a.nt ? 1 : 0);  // xcd: 0 plain, 1 chunked, 2 grouped
    if constexpr (Q == 27) {
        if (a.part != 0) return hipErrorInvalidValue;
        switch (key) {
            case 8: return a.aa ? aa_one<ST, COLL, WALLS, 1, 0, false, Q>(a, st)
                                : cs_one<ST, COLL, WALLS, 1, 0, false, Q>(a, st);
            case 10: return a.aa ? aa_one<ST, COLL, WALLS, 1, 1, false, Q>(a, st)
                                 : cs_one<ST, COLL, WALLS, 1, 1, false, Q>(a, st);
            default: return hipErrorInvalidValue;
        }
    } else {
        if (a.aa) {
            switch (key) {
                case 8: return aa_one<ST, COLL, WALLS, 1, 0, false, Q>(a, st);
                case 10: return aa_one<ST, COLL, WALLS, 1, 1, false, Q>(a, st);
                case 11: return aa_one<ST, COLL, WALLS, 1, 1, true, Q>(a, st);
                case 18: return aa_one<ST, COLL, WALLS, 2, 1, false, Q>(a, st);
                default: return hipErrorInvalidValue;
            }
        }
        if (a.part != 0) return cs_one<ST, COLL, WALLS, 1, 0, false, Q>(a, st);
        switch (key) {
            case 8: return cs_one<ST, COLL, WALLS, 1, 0, false, Q>(a, st);
            case 10: return cs_one<ST, COLL, WALLS, 1, 1, false, Q>(a, st);
            case 11: return cs_one<ST, COLL, WALLS, 1, 1, true, Q>(a, st);
            case 13: return cs_one<ST, COLL, WALLS, 1, 2, true, Q>(a, st);
            case 16: return cs_one<ST, COLL, WALLS, 2, 0, false, Q>(a, st);
            case 18: return cs_one<ST, COLL, WALLS, 2, 1, false, Q>(a, st);
            case 19: return cs_one<ST, COLL, WALLS, 2, 1, true, Q>(a, st);
            case 34: return cs_one<ST, COLL, WALLS, 4, 1, false, Q>(a, st);
            default: return hipErrorInvalidValue;
        }
    }
}

template <int ST, int COLL, int Q>
static hipError_t cs_walls(bool walls, const LaunchCS& a, hipStream_t st) {
    return walls ? cs_shape<ST, COLL, true, Q>(a, st) : cs_shape<ST, COLL, false, Q>(a, st);
}

template <int ST, int Q>
static hipError_t cs_coll(const LaunchCS& a, hipStream_t st) {
    switch (a.kp.collision) {
        case 0: return cs_walls<ST, 0, Q>(a.walls, a, st);
        case 1: return cs_walls<ST, 1, Q>(a.walls, a, st);
        default: return cs_walls<ST, 2, Q>(a.walls, a, st);
    }
}

template <int ST>
static hipError_t cs_lat(const LaunchCS& a, hipStream_t st) {
    return a.kp.q == 27 ? cs_coll<ST, 27>(a, st) : cs_coll<ST, 19>(a, st);
}

// row-wave kernel: D3Q19 only
template <int ST, int COLL, int K, bool NT>
static hipError_t rows_launch(bool walls, const LaunchCS& a, hipStream_t st) {
    using T = typename Store<ST>::T;
    const int rows = a.rows_ny * a.rows_nz;
    dim3 grid(a.part == 2 ? a.near_grid : (rows + 3) / 4), blk(256);
    if (grid.x == 0) return hipSuccess;
    if (walls)
        K1_LAUNCH((k_collide_stream_rows<ST, COLL, true, K, NT, 19>), grid, blk, st, a.boxes, a.rt, 0,
                  (const T*)a.fin, (T*)a.fout, a.kp, a.part, a.near_flags, a.near_list, a.near_count, a.near_epoch,
                  a.next_count, a.step_in, a.step_out);
    else
        K1_LAUNCH((k_collide_stream_rows<ST, COLL, false, K, NT, 19>), grid, blk, st, a.boxes, a.rt, 0,
                  (const T*)a.fin, (T*)a.fout, a.kp, a.part, a.near_flags, a.near_list, a.near_count, a.near_epoch,
                  a.next_count, a.step_in, a.step_out);
    return hipGetLastError();
}

template <int ST, int COLL>
static hipError_t rows_k(const LaunchCS& a, hipStream_t st) {
    const bool nt = a.variant == 2;
    switch (a.rows_k) {
        case 1: return nt ? rows_launch<ST, COLL, 1, true>(a.walls, a, st) : rows_launch<ST, COLL, 1, false>(a.walls, a, st);
        case 2: return nt ? rows_launch<ST, COLL, 2, true>(a.walls, a, st) : rows_launch<ST, COLL, 2, false>(a.walls, a, st);
        default: return nt ? rows_launch<ST, COLL, 4, true>(a.walls, a, st) : rows_launch<ST, COLL, 4, false>(a.walls, a, st);
    }
}

template <int ST>
static hipError_t rows_coll(const LaunchCS& a, hipStream_t st) {
    switch (a.kp.collision) {
        case 0: return rows_k<ST, 0>(a, st);
        case 1: return rows_k<ST, 1>(a, st);
        default: return rows_k<ST, 2>(a, st);
    }
}

hipError_t launch_collide_stream(const LaunchCS& a, hipStream_t st) {
    if (a.aa && (a.fin != a.fout || a.part != 0 || a.variant != 0)) return hipErrorInvalidValue;
    if (a.kp.q != 19 && a.kp.q != 27) return hipErrorInvalidValue;
    if (a.variant != 0 && a.rows_k > 0) {
        if (a.kp.q != 19) return hipErrorInvalidValue;
        switch (a.kp.storage) {
            case ST_F64: return rows_coll<ST_F64>(a, st);
            case ST_F32: return rows_coll<ST_F32>(a, st);
            case ST_F16: return rows_coll<ST_F16>(a, st);
            default: return rows_coll<ST_BF16>(a, st);
        }
    }
    switch (a.kp.storage) {
        case ST_F64: return cs_lat<ST_F64>(a, st);
        case ST_F32: return cs_lat<ST_F32>(a, st);
        case ST_F16: return cs_lat<ST_F16>(a, st);
        default: return cs_lat<ST_BF16>(a, st);
    }
}

#define LB_DISPATCH_ST(ST_VAR, CALL)                 \
    switch (ST_VAR) {                                \
        case ST_F64: { constexpr int SS = ST_F64; CALL; } break; \
        case ST_F32: { constexpr int SS = ST_F32; CALL; } break; \
        case ST_F16: { constexpr int SS = ST_F16; CALL; } break; \
        default: { constexpr int SS = ST_BF16; CALL; } break;    \
    }

hipError_t launch_init(const BoxDesc* boxes, const int* tile_box, int ntiles, void* f0, void* f1,
                       const int* box_init, const KParams& kp, hipStream_t st) {
    LB_DISPATCH_ST(kp.storage, {
        using T = typename Store<SS>::T;
        if (kp.q == 27)
            hipLaunchKernelGGL((k_init<SS, 27>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, (T*)f0, (T*)f1,
                               box_init, kp);
        else
            hipLaunchKernelGGL((k_init<SS, 19>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, (T*)f0, (T*)f1,
                               box_init, kp);
    });
    return hipGetLastError();
}

hipError_t launch_fields(const BoxDesc* boxes, int bi, const uint16_t* omap, const void* fin, int s0,
                         int count, double* out, const KParams& kp, hipStream_t st) {
    const int nb = (count + TILE - 1) / TILE;
    LB_DISPATCH_ST(kp.storage, {
        using T = typename Store<SS>::T;
        if (kp.q == 27)
            hipLaunchKernelGGL((k_fields<SS, 27>), dim3(nb), dim3(TILE), 0, st, boxes, bi, omap, (const T*)fin, s0,
                               count, out, kp);
        else
            hipLaunchKernelGGL((k_fields<SS, 19>), dim3(nb), dim3(TILE), 0, st, boxes, bi, omap, (const T*)fin, s0,
                               count, out, kp);
    });
    return hipGetLastError();
}

hipError_t launch_moments(const BoxDesc* boxes, int bi, int n, const uint16_t* omap, const void* fin,
                          double* partial, const KParams& kp, hipStream_t st) {
    const int nb = (n + TILE - 1) / TILE;
    LB_DISPATCH_ST(kp.storage, {
        using T = typename Store<SS>::T;
        if (kp.q == 27)
            hipLaunchKernelGGL((k_moments<SS, 27>), dim3(nb), dim3(TILE), 0, st, boxes, bi, omap, (const T*)fin,
                               partial, kp);
        else
            hipLaunchKernelGGL((k_moments<SS, 19>), dim3(nb), dim3(TILE), 0, st, boxes, bi, omap, (const T*)fin,
                               partial, kp);
    });
    return hipGetLastError();
}

hipError_t launch_box_energy(const BoxDesc* boxes, const int* tile_box, int ntiles, const uint16_t* omap,
                             const void* fin, const BoxMon* mon, double* partial, const KParams& kp, hipStream_t st) {
    LB_DISPATCH_ST(kp.storage, {
        using T = typename Store<SS>::T;
        if (kp.q == 27)
            hipLaunchKernelGGL((k_box_energy<SS, 27>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               (const T*)fin, mon, partial, kp);
        else
            hipLaunchKernelGGL((k_box_energy<SS, 19>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               (const T*)fin, mon, partial, kp);
    });
    return hipGetLastError();
}

hipError_t launch_relayout(const BoxDesc* boxes, const int* tile_box, int ntiles, const void* src, void* dst, int cs,
                           int cd, int storage, int q, hipStream_t st) {
    if (src == dst) return hipErrorInvalidValue;
    const int es = storage_bytes(storage);
    if (es == 8)
        hipLaunchKernelGGL((k_relayout<unsigned long long>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                           (const unsigned long long*)src, (unsigned long long*)dst, cs, cd, q);
    else if (es == 4)
        hipLaunchKernelGGL((k_relayout<uint32_t>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                           (const uint32_t*)src, (uint32_t*)dst, cs, cd, q);
    else
        hipLaunchKernelGGL((k_relayout<uint16_t>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                           (const uint16_t*)src, (uint16_t*)dst, cs, cd, q);
    return hipGetLastError();
}

hipError_t launch_poke(const BoxDesc* boxes, int bi, void* f, int s, int dir, double val, const KParams& kp,
                       hipStream_t st) {
    LB_DISPATCH_ST(kp.storage, {
        using T = typename Store<SS>::T;
        hipLaunchKernelGGL((k_poke<SS>), dim3(1), dim3(1), 0, st, boxes, bi, (T*)f, s, dir, val, kp);
    });
    return hipGetLastError();
}

}  // namespace lbd
