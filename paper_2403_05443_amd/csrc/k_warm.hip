// k_warm.hip - warm start of a run: the surrogate's inputs from the particle
// state, its outputs turned into particle velocities, and the fluid started
// from the creeping flow around each particle instead of from rest.
//
// Surrogate inputs (one thread per particle): with R(q) the body -> lab
// rotation, F_b = R^T F_ext, T_b = R^T T_ext, the equal-volume radius
// Req = (abc)^(1/3) and the load scale s = sqrt(|F_b|^2 + |T_b|^2 / Req^2):
//   x = (ln(a / sqrt(bc)), a / L, F_b / s, T_b / (Req s)),  L = (nx ny nz)^(1/3).
// Outputs y are the body-frame velocities in units of the Stokes scales:
//   U_b = y[0:3] s / (6 pi mu Req),  Omega_b = y[3:6] s / (8 pi mu Req^2).
//
// Start field (one thread per node): fluid nodes take the sum over the
// box's particles of the flow around a sphere of radius Req translating with
// U and rotating with Omega (Stokes' solution and the rotlet), at the
// minimum-image offset, minus the uniform velocity that makes the box's total
// momentum (fluid at rho0 plus particles) zero; nodes inside particle p move
// rigidly with it.  Every node gets the second-order equilibrium at rho0 and
// its velocity, written as pre-collision populations (slot (x - c_i, i)).
#include "lbell_dev.h"
#include "lbell_launch.h"

namespace lbd {

__device__ __forceinline__ void body_to_lab(const double q[4], double Rm[3][3]) {
    const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    Rm[0][0] = 1 - 2 * (q2 * q2 + q3 * q3);
    Rm[0][1] = 2 * (q1 * q2 - q0 * q3);
    Rm[0][2] = 2 * (q1 * q3 + q0 * q2);
    Rm[1][0] = 2 * (q1 * q2 + q0 * q3);
    Rm[1][1] = 1 - 2 * (q1 * q1 + q3 * q3);
    Rm[1][2] = 2 * (q2 * q3 - q0 * q1);
    Rm[2][0] = 2 * (q1 * q3 - q0 * q2);
    Rm[2][1] = 2 * (q2 * q3 + q0 * q1);
    Rm[2][2] = 1 - 2 * (q1 * q1 + q2 * q2);
}

__device__ __forceinline__ double eq_radius(const PartDev& P) { return cbrt(P.axes[0] * P.axes[1] * P.axes[2]); }

__global__ void k_warm_features(const BoxDesc* __restrict__ boxes, const PartDev* __restrict__ parts, int np,
                                float* __restrict__ X, double* __restrict__ s_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const PartDev& P = parts[p];
    const BoxDesc& B = boxes[P.box];
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    double Fb[3], Tb[3];
    for (int k = 0; k < 3; ++k) {
        Fb[k] = Rm[0][k] * P.Fext[0] + Rm[1][k] * P.Fext[1] + Rm[2][k] * P.Fext[2];
        Tb[k] = Rm[0][k] * P.Text[0] + Rm[1][k] * P.Text[1] + Rm[2][k] * P.Text[2];
    }
    const double R = eq_radius(P);
    const double s = sqrt(Fb[0] * Fb[0] + Fb[1] * Fb[1] + Fb[2] * Fb[2] +
                          (Tb[0] * Tb[0] + Tb[1] * Tb[1] + Tb[2] * Tb[2]) / (R * R));
    float* x = X + (long long)p * MLP_IN;
    x[0] = (float)log(P.axes[0] / sqrt(P.axes[1] * P.axes[2]));
    x[1] = (float)(P.axes[0] / cbrt((double)B.nx * B.ny * B.nz));
    for (int k = 0; k < 3; ++k) {
        x[2 + k] = s > 0 ? (float)(Fb[k] / s) : 0.f;
        x[5 + k] = s > 0 ? (float)(Tb[k] / (R * s)) : 0.f;
    }
    s_out[p] = s;
}

__global__ void k_warm_apply(PartDev* __restrict__ parts, int np, const float* __restrict__ Y,
                             const double* __restrict__ s_in, double mu, double* __restrict__ pred) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    PartDev& P = parts[p];
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    const double R = eq_radius(P), s = s_in[p];
    const double cu = s / (6.0 * M_PI * mu * R), cw = s / (8.0 * M_PI * mu * R * R);
    const float* y = Y + (long long)p * MLP_OUT;
    const double Ub[3] = {y[0] * cu, y[1] * cu, y[2] * cu}, Wb[3] = {y[3] * cw, y[4] * cw, y[5] * cw};
    for (int k = 0; k < 3; ++k) {
        P.U[k] = Rm[k][0] * Ub[0] + Rm[k][1] * Ub[1] + Rm[k][2] * Ub[2];
        P.W[k] = Rm[k][0] * Wb[0] + Rm[k][1] * Wb[1] + Rm[k][2] * Wb[2];
        pred[6 * p + k] = P.U[k];
        pred[6 * p + 3 + k] = P.W[k];
    }
}

// minimum-image offset of node (x, y, z) from the particle centre
__device__ __forceinline__ void offset(const PartDev& P, const BoxDesc& B, int x, int y, int z, double d[3]) {
    const int n[3] = {B.nx, B.ny, B.nz};
    const int c[3] = {x, y, z};
    for (int k = 0; k < 3; ++k) {
        double v = c[k] - P.xc[k];
        if (v >= 0.5 * n[k]) v -= n[k];
        if (v < -0.5 * n[k]) v += n[k];
        d[k] = v;
    }
}

// Velocity of node (x, y, z) of box bi before the mean correction: rigid
// motion inside a particle, else the sum of the particles' sphere fields.
__device__ void start_velocity(const BoxDesc& B, int bi, uint16_t owner, const PartDev* __restrict__ parts, int np,
                               int x, int y, int z, double u[3]) {
    u[0] = u[1] = u[2] = 0.0;
    if (owner != 0) {
        const PartDev& P = parts[owner - 1];
        double d[3];
        offset(P, B, x, y, z, d);
        u[0] = P.U[0] + P.W[1] * d[2] - P.W[2] * d[1];
        u[1] = P.U[1] + P.W[2] * d[0] - P.W[0] * d[2];
        u[2] = P.U[2] + P.W[0] * d[1] - P.W[1] * d[0];
        return;
    }
    for (int p = 0; p < np; ++p) {
        const PartDev& P = parts[p];
        if (P.box != bi) continue;
        double d[3];
        offset(P, B, x, y, z, d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double R = eq_radius(P);
        const double wx[3] = {P.W[1] * d[2] - P.W[2] * d[1], P.W[2] * d[0] - P.W[0] * d[2],
                              P.W[0] * d[1] - P.W[1] * d[0]};
        if (r < R) {  // fluid node inside the equal-volume sphere: rigid motion
            for (int k = 0; k < 3; ++k) u[k] += P.U[k] + wx[k];
            continue;
        }
        const double e[3] = {d[0] / r, d[1] / r, d[2] / r};
        const double Ue = P.U[0] * e[0] + P.U[1] * e[1] + P.U[2] * e[2];
        const double a1 = 0.75 * R / r, a3 = 0.25 * R * R * R / (r * r * r), rr = (R / r) * (R / r) * (R / r);
        for (int k = 0; k < 3; ++k)
            u[k] += a1 * (P.U[k] + Ue * e[k]) + a3 * (P.U[k] - 3.0 * Ue * e[k]) + rr * wx[k];
    }
}

// partial sums over the fluid nodes of each tile: sum of u (3) and the count
__global__ __launch_bounds__(TILE) void k_stokes_sum(const BoxDesc* __restrict__ boxes,
                                                     const int* __restrict__ tile_box,
                                                     const uint16_t* __restrict__ omap,
                                                     const PartDev* __restrict__ parts, int np,
                                                     double* __restrict__ partial) {
    __shared__ double red[4][TILE];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int bi = tile_box[tile];
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + tid;
    double v[4] = {0, 0, 0, 0};
    if (s < B.n && omap[B.ooff + s] == 0) {
        const int x = s % B.nx, t = s / B.nx, y = t % B.ny, z = t / B.ny;
        start_velocity(B, bi, 0, parts, np, x, y, z, v);
        v[3] = 1.0;
    }
    for (int k = 0; k < 4; ++k) red[k][tid] = v[k];
    __syncthreads();
    for (int h = TILE / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + h];
        __syncthreads();
    }
    if (tid < 4) partial[(long long)tile * 4 + tid] = red[tid][0];
}

// one thread per box: the uniform velocity removed from its fluid nodes
__global__ void k_stokes_mean(const BoxDesc* __restrict__ boxes, int nboxes, const PartDev* __restrict__ parts,
                              int np, const double* __restrict__ partial, double rho0, double* __restrict__ ubar) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nboxes) return;
    const BoxDesc& B = boxes[b];
    double S[4] = {0, 0, 0, 0};
    for (int t = B.tile0; t < B.tile0 + B.ntiles; ++t)
        for (int k = 0; k < 4; ++k) S[k] += partial[(long long)t * 4 + k];
    for (int p = 0; p < np; ++p)
        if (parts[p].box == b)
            for (int k = 0; k < 3; ++k) S[k] += parts[p].M * parts[p].U[k] / rho0;
    for (int k = 0; k < 3; ++k) ubar[3 * b + k] = S[3] > 0 ? S[k] / S[3] : 0.0;
}

template <int ST>
__global__ __launch_bounds__(TILE) void k_stokes_write(const BoxDesc* __restrict__ boxes,
                                                       const int* __restrict__ tile_box,
                                                       const uint16_t* __restrict__ omap,
                                                       const PartDev* __restrict__ parts, int np,
                                                       const double* __restrict__ ubar,
                                                       typename Store<ST>::T* __restrict__ f, KParams kp) {
    using S = Store<ST>;
    const int tile = blockIdx.x;
    const int bi = tile_box[tile];
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    const uint16_t owner = omap[B.ooff + s];
    if (owner == 0xFFFF) return;
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
    double u[3];
    start_velocity(B, bi, owner, parts, np, x, y, z, u);
    if (owner == 0)
        for (int k = 0; k < 3; ++k) u[k] -= ubar[3 * bi + k];
    const double rho0 = kp.rho0, uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    typename S::T* fb = f + B.foff;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double dev = wgt(i) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        // node (x, y, z) pulls f_i from slot (x - c_i, i)
        const int xs = wrap(x - cx(i), nx), ys = wrap(y - cy(i), ny), zs = wrap(z - cz(i), nz);
        const long long slot = xs + (long long)nx * (ys + (long long)ny * zs);
        S::st64(fb + (long long)i * B.stride + slot, dev, kp.scale);
    }
}

hipError_t launch_warm_features(const BoxDesc* boxes, const PartDev* parts, int np, float* X, double* s,
                                hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_features, dim3((np + 63) / 64), dim3(64), 0, st, boxes, parts, np, X, s);
    return hipGetLastError();
}

hipError_t launch_warm_apply(PartDev* parts, int np, const float* Y, const double* s, double mu, double* pred,
                             hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_apply, dim3((np + 63) / 64), dim3(64), 0, st, parts, np, Y, s, mu, pred);
    return hipGetLastError();
}

hipError_t launch_stokes_start(const BoxDesc* boxes, int nboxes, const int* tile_box, int ntiles,
                               const uint16_t* omap, const PartDev* parts, int np, double* partial, double* ubar,
                               void* f, const KParams& kp, hipStream_t st) {
    hipLaunchKernelGGL(k_stokes_sum, dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap, parts, np, partial);
    hipLaunchKernelGGL(k_stokes_mean, dim3((nboxes + 63) / 64), dim3(64), 0, st, boxes, nboxes, parts, np, partial,
                       kp.rho0, ubar);
    switch (kp.storage) {
        case ST_F64:
            hipLaunchKernelGGL((k_stokes_write<ST_F64>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               parts, np, ubar, (double*)f, kp);
            break;
        case ST_F32:
            hipLaunchKernelGGL((k_stokes_write<ST_F32>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               parts, np, ubar, (float*)f, kp);
            break;
        case ST_F16:
            hipLaunchKernelGGL((k_stokes_write<ST_F16>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               parts, np, ubar, (typename Store<ST_F16>::T*)f, kp);
            break;
        default:
            hipLaunchKernelGGL((k_stokes_write<ST_BF16>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap,
                               parts, np, ubar, (typename Store<ST_BF16>::T*)f, kp);
    }
    return hipGetLastError();
}

}  // namespace lbd
