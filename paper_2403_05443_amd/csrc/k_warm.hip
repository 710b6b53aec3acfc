// k_warm.hip - warm start of a run: the surrogate's inputs from the particle
// state, its outputs turned into particle velocities, and the fluid started
// from the creeping flow around each particle instead of from rest.
//
// Surrogate inputs (one thread per particle): with R(q) the body -> lab
// rotation, F_b = R^T F_ext, T_b = R^T T_ext, the equal-volume radius
// Req = (abc)^(1/3) and the load scale s = sqrt(|F_b|^2 + |T_b|^2 / Req^2):
//   x = (ln(a / sqrt(bc)), a / L, F_b / s, T_b / (Req s)),
// L = (nx ny nz / n)^(1/3), the box's volume per particle (n particles).
// Outputs y are the body-frame velocities in units of the Stokes scales:
//   U_b = y[0:3] s / (6 pi mu Req),  Omega_b = y[3:6] s / (8 pi mu Req^2).
// A squirmer carries no load of its own; it enters with the equivalent
// propulsive force along its axis (body x), the drag of a prolate spheroid
// translating along its axis at the free swimming speed of eq. squirmervel:
//   F_eff = 6 pi mu a X^A(e) U_s,  U_s = B1 e^-1 (e^-1 - (e^-2 - 1) arcoth(1/e)),
// e = sqrt(1 - b^2 / a^2), X^A(e) = (8/3) e^3 / (-2 e + (1 + e^2) ln((1+e)/(1-e)))
// (the sphere's limits 1 and 2 B1 / 3 for e -> 0), added to F_b.
//
// Start field: the creeping flow the particles' loads drive in the periodic
// box.  Per node, the sum over the box's particles of the free-space flow
// and pressure that the particle's load drives (particle_flow: the exact
// flow of a prolate spheroid, else that of the equal-volume sphere;
// minimum-image offsets, rigid inside the body), computed once per node
// (k_stokes_free) -- whose Fourier modes |n_i| <= 2 are replaced by those of
// the periodic solution of the same loads (the force spread as the traction
// on the translating ellipsoid, the torque as that on the rotating prolate
// spheroid, or over the sphere of radius Req for other bodies),
// so the box's slowest shear modes start at their steady values.  A fluid
// node's density carries the pressure, rho = rho0 + (p - pbar) / c_s^2 (pbar
// the fluid's mean: the mass is unchanged; without it the pressure builds up
// through sound waves that ring in the box for hundreds of steps), and the
// uniform velocity that makes the box's total momentum (fluid sum rho u plus
// particles) zero is removed; nodes inside particle p have rho0 and move
// rigidly with its U, Omega.  Every node gets the second-order equilibrium
// at its density and velocity, written as pre-collision populations (slot
// (x - c_i, i)).
#include <type_traits>

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

// Equivalent propulsive force of a squirmer along its body x axis (0 for a
// passive particle); a prolate spheroid, b taken as sqrt(bc).  Below
// e = 1e-3 the sphere's limits hold to 1e-6.
__device__ double propulsive_force(const PartDev& P, double mu) {
    if (P.B1 == 0.0) return 0.0;
    const double a = P.axes[0], b = sqrt(P.axes[1] * P.axes[2]);
    const double e = a > b ? sqrt(1.0 - (b / a) * (b / a)) : 0.0;
    double XA = 1.0, Us = 2.0 * P.B1 / 3.0;
    if (e >= 1e-3) {
        const double lg = log((1.0 + e) / (1.0 - e));
        XA = (8.0 / 3.0) * e * e * e / (-2.0 * e + (1.0 + e * e) * lg);
        Us = P.B1 / e * (1.0 / e - (1.0 / (e * e) - 1.0) * 0.5 * lg);
    }
    return 6.0 * M_PI * mu * a * XA * Us;
}

__global__ void k_warm_features(const BoxDesc* __restrict__ boxes, const PartDev* __restrict__ parts, int np,
                                double mu, float* __restrict__ X, double* __restrict__ s_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const PartDev& P = parts[p];
    const BoxDesc& B = boxes[P.box];
    int nbox = 0;  // the box's particles (a one-off pass; np is at most 65534)
    for (int k = 0; k < np; ++k) nbox += parts[k].box == P.box;
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    double Fb[3], Tb[3];
    for (int k = 0; k < 3; ++k) {
        Fb[k] = Rm[0][k] * P.Fext[0] + Rm[1][k] * P.Fext[1] + Rm[2][k] * P.Fext[2];
        Tb[k] = Rm[0][k] * P.Text[0] + Rm[1][k] * P.Text[1] + Rm[2][k] * P.Text[2];
    }
    Fb[0] += propulsive_force(P, mu);
    const double R = eq_radius(P);
    const double s = sqrt(Fb[0] * Fb[0] + Fb[1] * Fb[1] + Fb[2] * Fb[2] +
                          (Tb[0] * Tb[0] + Tb[1] * Tb[1] + Tb[2] * Tb[2]) / (R * R));
    float* x = X + (long long)p * MLP_IN;
    x[0] = (float)log(P.axes[0] / sqrt(P.axes[1] * P.axes[2]));
    x[1] = (float)(P.axes[0] / cbrt((double)B.nx * B.ny * B.nz / nbox));
    for (int k = 0; k < 3; ++k) {
        x[2 + k] = s > 0 ? (float)(Fb[k] / s) : 0.f;
        x[5 + k] = s > 0 ? (float)(Tb[k] / (R * s)) : 0.f;
    }
    s_out[p] = s;
}

__global__ void k_warm_apply(PartDev* __restrict__ parts, int np, const float* __restrict__ Y,
                             const double* __restrict__ s_in, double mu, double* __restrict__ pred, int only_box) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    PartDev& P = parts[p];
    if (only_box >= 0 && P.box != only_box) return;
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    const double R = eq_radius(P), s = s_in[p];
    const double cu = s / (6.0 * M_PI * mu * R), cw = s / (8.0 * M_PI * mu * R * R);
    const float* y = Y + (long long)p * MLP_OUT;
    double Ub[3] = {y[0] * cu, y[1] * cu, y[2] * cu}, Wb[3] = {y[3] * cw, y[4] * cw, y[5] * cw};
    {  // a prediction above the surface-speed limit of the solve is scaled down to it
        const double amax = fmax(P.axes[0], fmax(P.axes[1], P.axes[2]));
        const double sp = sqrt(Ub[0] * Ub[0] + Ub[1] * Ub[1] + Ub[2] * Ub[2]) +
                          sqrt(Wb[0] * Wb[0] + Wb[1] * Wb[1] + Wb[2] * Wb[2]) * amax;
        if (!(sp <= 0.5)) {
            const double f = sp > 0.5 && sp <= 1e300 ? 0.5 / sp : 0.0;  // a non-finite prediction becomes rest
            for (int k = 0; k < 3; ++k) {
                Ub[k] = f == 0.0 ? 0.0 : Ub[k] * f;
                Wb[k] = f == 0.0 ? 0.0 : Wb[k] * f;
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        P.U[k] = Rm[k][0] * Ub[0] + Rm[k][1] * Ub[1] + Rm[k][2] * Ub[2];
        P.W[k] = Rm[k][0] * Wb[0] + Rm[k][1] * Wb[1] + Rm[k][2] * Wb[2];
        pred[6 * p + k] = P.U[k];
        pred[6 * p + 3 + k] = P.W[k];
    }
}

// Normalised body-frame response of every particle at its current
// velocities (the training target of the surrogate; inverse of k_warm_apply).
__global__ void k_warm_targets(const PartDev* __restrict__ parts, int np, const double* __restrict__ s_in,
                               double mu, float* __restrict__ Y) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const PartDev& P = parts[p];
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    const double R = eq_radius(P), s = s_in[p];
    const double cu = s > 0 ? 6.0 * M_PI * mu * R / s : 0.0, cw = s > 0 ? 8.0 * M_PI * mu * R * R / s : 0.0;
    float* y = Y + (long long)p * MLP_OUT;
    for (int k = 0; k < 3; ++k) {
        y[k] = (float)(cu * (Rm[0][k] * P.U[0] + Rm[1][k] * P.U[1] + Rm[2][k] * P.U[2]));
        y[3 + k] = (float)(cw * (Rm[0][k] * P.W[0] + Rm[1][k] * P.W[1] + Rm[2][k] * P.W[2]));
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

constexpr int WK = 2;                  // modes |n_i| <= WK carry the periodic correction
constexpr int WM = (2 * WK + 1) * (2 * WK + 1) * (2 * WK + 1);  // mode slots per box (index 62 = n = 0)

__device__ __forceinline__ int wk_axis(int L) { return min(WK, (L - 1) / 2); }

// Gauss-Legendre rules on [-1, 1] of 24, 16 and 12 points, one table: the
// positive nodes and their weights of each (the rules are symmetric), at
// rows 0, 12 and 20.
__constant__ double GLTAB[26][2] = {
    {0.06405689286260563, 0.12793819534675221}, {0.1911188674736163, 0.1258374563468283},
    {0.3150426796961634, 0.12167047292780342},  {0.4337935076260451, 0.11550566805372561},
    {0.5454214713888396, 0.1074442701159656},   {0.6480936519369755, 0.09761865210411406},
    {0.7401241915785544, 0.08619016153195329},  {0.820001985973903, 0.07334648141108041},
    {0.886415527004401, 0.05929858491543674},   {0.9382745520027328, 0.04427743881741955},
    {0.9747285559713095, 0.028531388628933743}, {0.9951872199970213, 0.012341229799987091},
    {0.09501250983763745, 0.18945061045506859}, {0.2816035507792589, 0.1826034150449236},
    {0.45801677765722737, 0.16915651939500262}, {0.6178762444026438, 0.14959598881657676},
    {0.755404408355003, 0.12462897125553403},   {0.8656312023878318, 0.09515851168249259},
    {0.9445750230732326, 0.062253523938647706}, {0.9894009349916499, 0.027152459411754037},
    {0.1252334085114689, 0.2491470458134027},   {0.3678314989981802, 0.23349253653835464},
    {0.5873179542866175, 0.20316742672306565},  {0.7699026741943047, 0.1600783285433461},
    {0.9041172563704748, 0.10693932599531888},  {0.9815606342467192, 0.04717533638651202},
};

// Below this eccentricity a prolate spheroid's flow is taken as the sphere's
// (the two differ by O(e^2)).
constexpr double E_LINE = 1e-4;
constexpr int UF = 4;  // doubles per node of the staged free field: velocity, pressure
constexpr int MC = 8;  // doubles per mode: (re, im) of velocity and pressure
constexpr int NPART = 8;  // partial sums per tile of k_stokes_sum

__device__ __forceinline__ bool loaded(const PartDev& P) {
    return P.Fext[0] != 0.0 || P.Fext[1] != 0.0 || P.Fext[2] != 0.0 || P.Text[0] != 0.0 || P.Text[1] != 0.0 ||
           P.Text[2] != 0.0;
}

// Free-space creeping flow that the load of particle P drives, added to
// (u[0..2], u[3]) = (velocity, pressure) at offset d from its centre; rigid
// motion and no pressure inside the body.  The pressure is that of the
// Stokeslets, 2 mu (s.r) / R^3, and of the stresslets, 2 mu (r.p)(r.m) / R^5
// times theirs; the potential singularities and the rotlets carry none
// (the sphere: 3 mu R (U.d) / (2 r^3) = F.d / (4 pi r^3)).
//
// Prolate spheroid (a > b = c): the exact solution of Chwang & Wu (J. Fluid
// Mech. 63, 1974; 67, 1975) as singularities on the focal segment |xi| <= f,
// f = a e, axis p, g(xi) = f^2 - xi^2, r = d - xi p, R = |r|; with
// s = F / (16 pi mu f) and t = T / (8 pi mu (4/3) f^3), t_c its part across p:
//   Stokeslets s / R + (s.r) r / R^3 (uniform: they carry the force),
//   potential dipoles -(1 - e^2) / (2 e^2) g [-s / R^3 + 3 (s.r) r / R^5],
//   rotlets g t x r / R^3 (they carry the torque),
//   stresslets 3 e^2 / (2 - e^2) g r (r.p)(r.m) / R^5, m = t_c x p,
//   potential quadrupoles (1 - e^2) / (4 (2 - e^2)) g^2 (p.grad) of the
//   dipole of m: 3 (m (r.p) + (r.m) p) / R^5 - 15 (r.m)(r.p) r / R^7.
// The body moves with the velocities of eq. drag4's X^A, Y^A, X^C, Y^C:
// V = F_p / (16 pi mu f alpha_p) + F_c / (16 pi mu f alpha_c), alpha_p =
// e^2 / D1, alpha_c = 2 e^2 / D2; Omega = t_p D3 / (1 - e^2) + t_c D1 /
// (2 - e^2); D1 = -2e + (1 + e^2) L, D2 = 2e + (3e^2 - 1) L, D3 = 2e -
// (1 - e^2) L, L = ln((1 + e) / (1 - e)) (power series below e = 1/2, where
// they cancel).  The segment integrals are taken with the substitution
// xi = xi0 -+ delta sinh(t) about the point xi0 of the segment nearest d
// (delta the distance to it), which smooths the near-tip peaks, and
// Gauss-Legendre points on each side of xi0: 24 within delta < f / 2, 16
// within delta < 3 f / 2, 12 beyond (each within ~2e-15 of the integral,
// relative to the velocity, measured against adaptive quadrature).
// Every other shape: the sphere of radius Req = (abc)^(1/3) moving with
// F / (6 pi mu Req) and turning with T / (8 pi mu Req^3) (Stokes' solution
// and the rotlet), rigid inside Req.
__device__ void particle_flow(const PartDev& P, double mu, const double d[3], double u[4]) {
    const double a = P.axes[0], b = P.axes[1];
    const double e2 = a > b && b == P.axes[2] ? 1.0 - (b / a) * (b / a) : 0.0;
    if (e2 < E_LINE * E_LINE) {
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double R = eq_radius(P);
        const double cu = 1.0 / (6.0 * M_PI * mu * R), cw = 1.0 / (8.0 * M_PI * mu * R * R * R);
        const double U[3] = {P.Fext[0] * cu, P.Fext[1] * cu, P.Fext[2] * cu};
        const double W[3] = {P.Text[0] * cw, P.Text[1] * cw, P.Text[2] * cw};
        const double wx[3] = {W[1] * d[2] - W[2] * d[1], W[2] * d[0] - W[0] * d[2], W[0] * d[1] - W[1] * d[0]};
        if (r < R) {
            for (int k = 0; k < 3; ++k) u[k] += U[k] + wx[k];
            return;
        }
        const double ex[3] = {d[0] / r, d[1] / r, d[2] / r};
        const double Ue = U[0] * ex[0] + U[1] * ex[1] + U[2] * ex[2];
        const double a1 = 0.75 * R / r, a3 = 0.25 * R * R * R / (r * r * r), rr = (R / r) * (R / r) * (R / r);
        for (int k = 0; k < 3; ++k)
            u[k] += a1 * (U[k] + Ue * ex[k]) + a3 * (U[k] - 3.0 * Ue * ex[k]) + rr * wx[k];
        u[3] += 1.5 * mu * R * Ue / (r * r);
        return;
    }
    const double e = sqrt(e2), f = a * e;
    double D1 = 0.0, D2 = 0.0, D3 = 0.0;
    if (e < 0.5) {  // D1 = sum 8k e^(2k+1) / (4k^2 - 1), D2 = sum 8(k+1) ..., D3 = sum 4 ... (k >= 1)
        double ek = e * e2;
        for (int k = 1; k <= 30; ++k) {
            const double den = 4.0 * k * k - 1.0;
            D1 += 8.0 * k * ek / den;
            D2 += 8.0 * (k + 1) * ek / den;
            D3 += 4.0 * ek / den;
            ek *= e2;
        }
    } else {
        const double L = log((1.0 + e) / (1.0 - e));
        D1 = -2.0 * e + (1.0 + e2) * L;
        D2 = 2.0 * e + (3.0 * e2 - 1.0) * L;
        D3 = 2.0 * e - (1.0 - e2) * L;
    }
    const double bfac = -(1.0 - e2) / (2.0 * e2), dl = 3.0 * e2 / (2.0 - e2), ka = (1.0 - e2) / (4.0 * (2.0 - e2));
    double Rm[3][3];
    body_to_lab(P.q, Rm);
    const double p[3] = {Rm[0][0], Rm[1][0], Rm[2][0]};
    const double Fp = P.Fext[0] * p[0] + P.Fext[1] * p[1] + P.Fext[2] * p[2];
    const double Tp = P.Text[0] * p[0] + P.Text[1] * p[1] + P.Text[2] * p[2];
    const double cf = 1.0 / (16.0 * M_PI * mu * f), ct = 1.0 / (8.0 * M_PI * mu * (4.0 / 3.0) * f * f * f);
    double U[3], W[3], S1[3], G[3], Gc[3];
    for (int k = 0; k < 3; ++k) {
        S1[k] = P.Fext[k] * cf;
        G[k] = P.Text[k] * ct;
        Gc[k] = (P.Text[k] - Tp * p[k]) * ct;
        U[k] = Fp * p[k] * cf * D1 / e2 + (P.Fext[k] - Fp * p[k]) * cf * D2 / (2.0 * e2);
        W[k] = Tp * p[k] * ct * D3 / (1.0 - e2) + Gc[k] * D1 / (2.0 - e2);
    }
    const double m[3] = {Gc[1] * p[2] - Gc[2] * p[1], Gc[2] * p[0] - Gc[0] * p[2], Gc[0] * p[1] - Gc[1] * p[0]};
    const double z = d[0] * p[0] + d[1] * p[1] + d[2] * p[2];
    const double rho2 = fmax(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - z * z, 0.0);
    if (z * z / (a * a) + rho2 / (b * b) < 1.0) {  // inside: rigid motion
        u[0] += U[0] + W[1] * d[2] - W[2] * d[1];
        u[1] += U[1] + W[2] * d[0] - W[0] * d[2];
        u[2] += U[2] + W[0] * d[1] - W[1] * d[0];
        return;
    }
    const double x0 = fmin(fmax(z, -f), f);
    const double delta = sqrt(rho2 + (z - x0) * (z - x0));  // > 0: the segment lies inside the body
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ng = delta < 0.5 * f ? 24 : delta < 1.5 * f ? 16 : 12, half = ng / 2;
    const int row = ng == 24 ? 0 : ng == 16 ? 12 : 20;
    for (int side = 0; side < 2; ++side) {
        const double sgn = side ? 1.0 : -1.0, len = side ? f - x0 : x0 + f;
        if (len <= 0.0) continue;
        const double tm = asinh(len / delta);
        for (int j = 0; j < ng; ++j) {
            const int ri = row + (j < half ? half - 1 - j : j - half);
            const double tj = j < half ? -GLTAB[ri][0] : GLTAB[ri][0], wj = GLTAB[ri][1];
            const double t = 0.5 * tm * (tj + 1.0), et = exp(t), it = 1.0 / et;
            const double xi = x0 + sgn * delta * 0.5 * (et - it);
            const double wq = 0.5 * tm * wj * delta * 0.5 * (et + it);
            const double r[3] = {d[0] - xi * p[0], d[1] - xi * p[1], d[2] - xi * p[2]};
            const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            const double iR = rsqrt(R2), iR2 = iR * iR, iR3 = iR * iR2, iR5 = iR3 * iR2, iR7 = iR5 * iR2;
            const double g = (f - xi) * (f + xi);
            const double Sr = S1[0] * r[0] + S1[1] * r[1] + S1[2] * r[2];
            const double rp = r[0] * p[0] + r[1] * p[1] + r[2] * p[2];
            const double rm = r[0] * m[0] + r[1] * m[1] + r[2] * m[2];
            const double Gxr[3] = {G[1] * r[2] - G[2] * r[1], G[2] * r[0] - G[0] * r[2], G[0] * r[1] - G[1] * r[0]};
            const double cS = bfac * g, cQ = ka * g * g;
            for (int k = 0; k < 3; ++k) {
                const double v = S1[k] * iR + Sr * r[k] * iR3                      // Stokeslets
                                 + cS * (-S1[k] * iR3 + 3.0 * Sr * r[k] * iR5)     // potential dipoles
                                 + g * Gxr[k] * iR3                                // rotlets
                                 + dl * g * r[k] * rp * rm * iR5                   // stresslets
                                 + cQ * (3.0 * (m[k] * rp + rm * p[k]) * iR5 - 15.0 * rm * rp * r[k] * iR7);
                acc[k] += wq * v;
            }
            acc[3] += wq * 2.0 * mu * (Sr * iR3 + dl * g * rp * rm * iR5);
        }
    }
    for (int k = 0; k < 4; ++k) u[k] += acc[k];
}

// Free-space flow and pressure of every node of the started boxes (the sum
// over each box's loaded particles of particle_flow), node-major into uf at
// UF * (ooff + site - base).  A work-group per tile; the box's loaded particles
// are listed in index order, TILE at a time, in LDS.
__global__ __launch_bounds__(TILE) void k_stokes_free(const BoxDesc* __restrict__ boxes,
                                                      const int* __restrict__ tile_box,
                                                      const PartDev* __restrict__ parts, int np, double mu,
                                                      int only_box, long long base, double* __restrict__ uf) {
    __shared__ int list[TILE];
    __shared__ int wcnt[TILE / 64];
    const int tile = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int bi = tile_box[tile];
    if (only_box >= 0 && bi != only_box) return;  // uniform over the block
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + tid;
    const int x = s % B.nx, t = s / B.nx, y = t % B.ny, z = t / B.ny;
    double u[UF] = {0.0, 0.0, 0.0, 0.0};
    for (int p0 = 0; p0 < np; p0 += TILE) {
        const int p = p0 + tid;
        const bool take = p < np && parts[p].box == bi && loaded(parts[p]);
        const unsigned long long bal = __ballot(take);
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, cnt = 0;
        for (int w = 0; w < TILE / 64; ++w) {
            off += w < wv ? wcnt[w] : 0;
            cnt += wcnt[w];
        }
        if (take) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = p;
        __syncthreads();
        if (s < B.n)
            for (int j = 0; j < cnt; ++j) {
                const PartDev& P = parts[list[j]];
                double d[3];
                offset(P, B, x, y, z, d);
                particle_flow(P, mu, d, u);
            }
        __syncthreads();
    }
    if (s < B.n) {
        double* o = uf + UF * (B.ooff + s - base);
        for (int k = 0; k < UF; ++k) o[k] = u[k];
    }
}

// Periodic correction Re sum_m c_m exp(i k_m . x) at node (x, y, z); c: the
// box's WM x 3 complex coefficients (re, im), zero for unused slots.
// exp(i 2 pi n x / L) for n = -WK..WK (WK = 2) into e[n + WK] (re, im):
// powers of the n = 1 term, the negative ones conjugate.
static_assert(WK == 2, "twiddles() builds the modes |n| <= 2");
__device__ __forceinline__ void powers(double c1, double s1, double e[2 * WK + 1][2]) {
    const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * s1 * c1;
    e[WK][0] = 1.0;
    e[WK][1] = 0.0;
    e[WK + 1][0] = c1;
    e[WK + 1][1] = s1;
    e[WK - 1][0] = c1;
    e[WK - 1][1] = -s1;
    e[WK + 2][0] = c2;
    e[WK + 2][1] = s2;
    e[WK - 2][0] = c2;
    e[WK - 2][1] = -s2;
}

__device__ __forceinline__ void twiddles(int x, int L, double e[2 * WK + 1][2]) {
    double s1, c1;
    sincospi(2.0 * x / L, &s1, &c1);
    powers(c1, s1, e);
}

// The periodic correction Re sum_m c_m exp(i k_m . x) at the nodes of one
// tile, in two stages.  row_coefs (every thread of the work-group calls it):
// for each row (y, z) the tile touches, R[a][k] = sum over (ny, nz) of
// c_(a, ny, nz)[k] exp(i (ky y + kz z)) into LDS (slots outside the box's
// mode set hold c = 0); then a node's correction is Re sum_a R[a][k]
// exp(i kx x) (start_velocity).  c: the box's WM x MC coefficients.
constexpr int CROWS = TILE / 4 + 2;  // rows a tile can touch (edges are at least 4)
struct RowCoefs {
    double tw[CROWS][2][2 * WK + 1][2];  // exp(i 2 pi n y / ny), exp(i 2 pi n z / nz) of each row
    double R[CROWS][2 * WK + 1][UF][2];
    int row0;
};

__device__ void row_coefs(const BoxDesc& B, const double* __restrict__ c, int s0, RowCoefs& rc) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int row0 = s0 / B.nx, nrows = (min(s0 + TILE, B.n) - 1) / B.nx - row0 + 1;
    if (tid == 0) rc.row0 = row0;
    for (int r = tid; r < nrows; r += nt) {
        const int row = row0 + r;
        twiddles(row % B.ny, B.ny, rc.tw[r][0]);
        twiddles(row / B.ny, B.nz, rc.tw[r][1]);
    }
    __syncthreads();
    for (int t = tid; t < nrows * (2 * WK + 1) * UF; t += nt) {
        const int r = t / ((2 * WK + 1) * UF), a = (t / UF) % (2 * WK + 1), k = t % UF;
        double re = 0.0, im = 0.0;
        for (int iz = 0; iz < 2 * WK + 1; ++iz) {
            const double cz = rc.tw[r][1][iz][0], sz = rc.tw[r][1][iz][1];
            for (int iy = 0; iy < 2 * WK + 1; ++iy) {
                const double cy = rc.tw[r][0][iy][0], sy = rc.tw[r][0][iy][1];
                const double er = cy * cz - sy * sz, ei = sy * cz + cy * sz;  // exp(i (ky y + kz z))
                const double* cm = c + MC * (a + (2 * WK + 1) * (iy + (2 * WK + 1) * iz));
                re += cm[2 * k] * er - cm[2 * k + 1] * ei;
                im += cm[2 * k] * ei + cm[2 * k + 1] * er;
            }
        }
        rc.R[r][a][k][0] = re;
        rc.R[r][a][k][1] = im;
    }
    __syncthreads();
}

// Velocity and pressure of site s = (x, y, z) of box B before the mean
// corrections: rigid motion and no pressure inside a particle, else the
// corrected load-driven flow (uf: the free flow of k_stokes_free; rc: the
// tile's row_coefs).
__device__ void start_velocity(const BoxDesc& B, uint16_t owner, const PartDev* __restrict__ parts,
                               const double* __restrict__ uf, long long base, const RowCoefs& rc, int s, int x,
                               int y, int z, double u[UF]) {
    if (owner != 0) {
        const PartDev& P = parts[owner - 1];
        double d[3];
        offset(P, B, x, y, z, d);
        u[0] = P.U[0] + P.W[1] * d[2] - P.W[2] * d[1];
        u[1] = P.U[1] + P.W[2] * d[0] - P.W[0] * d[2];
        u[2] = P.U[2] + P.W[0] * d[1] - P.W[1] * d[0];
        u[3] = 0.0;
        return;
    }
    const double* o = uf + UF * (B.ooff + s - base);
    for (int k = 0; k < UF; ++k) u[k] = o[k];
    double ex[2 * WK + 1][2];
    twiddles(x, B.nx, ex);
    const int r = s / B.nx - rc.row0;
    for (int a = 0; a < 2 * WK + 1; ++a)
        for (int k = 0; k < UF; ++k) u[k] += rc.R[r][a][k][0] * ex[a][0] - rc.R[r][a][k][1] * ex[a][1];
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Discrete Fourier sums S_m = sum_x (u, p)_free(x) exp(-i k_m . x) over every
// node of a box, for the modes of one (ny, nz) pair and all nx: work-group
// 25 b + g takes box b and pair g, so the 25 work-groups of a box run
// together and stream its staged field through the caches about once.
// Edges up to TW_MAX take their phase factors from tables in LDS.
constexpr int TW_MAX = 1024;
__global__ __launch_bounds__(256) void k_stokes_modes(const BoxDesc* __restrict__ boxes,
                                                      const double* __restrict__ uf, long long base, int only_box,
                                                      double* __restrict__ S) {
    __shared__ double red[4][2 * WK + 1][MC];
    __shared__ double tw[3][TW_MAX][2];  // exp(i 2 pi x / nx), exp(i 2 pi ny' y / ny), exp(i 2 pi nz' z / nz)
    const int g = blockIdx.x % ((2 * WK + 1) * (2 * WK + 1)), bi = blockIdx.x / ((2 * WK + 1) * (2 * WK + 1));
    if (only_box >= 0 && bi != only_box) return;  // uniform over the block
    const BoxDesc& B = boxes[bi];
    const int ny_ = g % (2 * WK + 1) - WK, nz_ = g / (2 * WK + 1) - WK;
    const int Kx = wk_axis(B.nx), Ky = wk_axis(B.ny), Kz = wk_axis(B.nz);
    if (abs(ny_) > Ky || abs(nz_) > Kz) return;  // uniform over the block
    const bool tab = B.nx <= TW_MAX && B.ny <= TW_MAX && B.nz <= TW_MAX;
    if (tab) {
        for (int i = threadIdx.x; i < B.nx; i += blockDim.x) sincospi(2.0 * i / B.nx, &tw[0][i][1], &tw[0][i][0]);
        for (int i = threadIdx.x; i < B.ny; i += blockDim.x)
            sincospi(2.0 * ny_ * i / B.ny, &tw[1][i][1], &tw[1][i][0]);
        for (int i = threadIdx.x; i < B.nz; i += blockDim.x)
            sincospi(2.0 * nz_ * i / B.nz, &tw[2][i][1], &tw[2][i][0]);
    }
    __syncthreads();
    double acc[2 * WK + 1][MC];
#pragma unroll
    for (int a = 0; a < 2 * WK + 1; ++a)
#pragma unroll
        for (int k = 0; k < MC; ++k) acc[a][k] = 0.0;
    for (int s = threadIdx.x; s < B.n; s += blockDim.x) {
        const int x = s % B.nx, t = s / B.nx, y = t % B.ny, z = t / B.ny;
        const double* o = uf + UF * (B.ooff + s - base);
        const double u[UF] = {o[0], o[1], o[2], o[3]};
        double syz, cyz, ex[2 * WK + 1][2];
        if (tab) {
            cyz = tw[1][y][0] * tw[2][z][0] - tw[1][y][1] * tw[2][z][1];
            syz = tw[1][y][1] * tw[2][z][0] + tw[1][y][0] * tw[2][z][1];
            powers(tw[0][x][0], tw[0][x][1], ex);
        } else {
            sincospi(2.0 * ((double)ny_ * y / B.ny + (double)nz_ * z / B.nz), &syz, &cyz);
            twiddles(x, B.nx, ex);
        }
#pragma unroll
        for (int nx = -WK; nx <= WK; ++nx) {  // fixed trip count: the accumulators stay in registers
            if (nx < -Kx || nx > Kx) continue;
            const double cx_ = ex[nx + WK][0], sx = ex[nx + WK][1];
            // exp(-i theta) = cos theta - i sin theta, theta = kx x + ky y + kz z
            const double c = cx_ * cyz - sx * syz, sn = sx * cyz + cx_ * syz;
#pragma unroll
            for (int k = 0; k < UF; ++k) {
                acc[nx + WK][2 * k] += u[k] * c;
                acc[nx + WK][2 * k + 1] -= u[k] * sn;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 2 * WK + 1; ++a)
#pragma unroll
        for (int k = 0; k < MC; ++k) {
            const double v = wave_sum(acc[a][k]);
            if (lane == 0) red[wv][a][k] = v;
        }
    __syncthreads();
    if (threadIdx.x < (2 * WK + 1) * MC) {
        const int a = threadIdx.x / MC, k = threadIdx.x % MC;
        const double v = red[0][a][k] + red[1][a][k] + red[2][a][k] + red[3][a][k];
        const int m = a + (2 * WK + 1) * ((ny_ + WK) + (2 * WK + 1) * (nz_ + WK));
        S[((long long)bi * WM + m) * MC + k] = v;
    }
}

// Correction coefficients: one thread per (box, mode slot): the periodic
// solution's coefficient of every particle of the box minus the free flow's
// DFT coefficient S_m / N; zero for slots outside the box's mode set.  The
// pressure's is -i (k.f) / k^2 of the force density f (the torque's has no
// divergence and drives none).
__global__ void k_stokes_coef(const BoxDesc* __restrict__ boxes, int nboxes, const PartDev* __restrict__ parts,
                              int np, double mu, const double* __restrict__ S, double* __restrict__ C) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nboxes * WM) return;
    const int bi = id / WM, m = id % WM;
    const BoxDesc& B = boxes[bi];
    const int n[3] = {m % (2 * WK + 1) - WK, (m / (2 * WK + 1)) % (2 * WK + 1) - WK, m / ((2 * WK + 1) * (2 * WK + 1)) - WK};
    const int L[3] = {B.nx, B.ny, B.nz};
    double* c = C + (long long)id * MC;
    bool use = !(n[0] == 0 && n[1] == 0 && n[2] == 0);
    for (int a = 0; a < 3; ++a) use = use && abs(n[a]) <= wk_axis(L[a]);
    for (int k = 0; k < MC; ++k) c[k] = 0.0;
    if (!use) return;
    const double V = (double)B.n;
    double k[3];
    for (int a = 0; a < 3; ++a) k[a] = 2.0 * M_PI * n[a] / L[a];
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    for (int p = 0; p < np; ++p) {
        const PartDev& P = parts[p];
        if (P.box != bi) continue;
        // The traction of a body in rigid motion is sigma(x) (F + C x), sigma
        // the unit sphere's uniform layer mapped onto the surface: for an
        // ellipsoid (diag(a, b, c) in the body frame) its transform is
        // F sinc(kappa) - 3 i (Q^T k) j1(kappa) / kappa, kappa = |diag(a, b, c)
        // R^T k|, Q = integral of x f^T the first moment: the torque's
        // antisymmetric part, Q^T k = -(k x T) / 2, and for a prolate spheroid
        // the line solution's stresslet e^2 / (2 - e^2) sym(p (T_c x p)).
        // The force is spread on every ellipsoid so; the torque on the
        // prolate spheroid so and on any other body over the sphere of
        // radius Req (kappa = |k| Req, no stresslet).
        double Rm[3][3];
        body_to_lab(P.q, Rm);
        double ka2 = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double kb = (k[0] * Rm[0][j] + k[1] * Rm[1][j] + k[2] * Rm[2][j]) * P.axes[j];
            ka2 += kb * kb;
        }
        const double xa = sqrt(ka2), sinc = sin(xa) / xa;
        const double kF = k[0] * P.Fext[0] + k[1] * P.Fext[1] + k[2] * P.Fext[2];
        double g[3] = {-0.5 * (k[1] * P.Text[2] - k[2] * P.Text[1]), -0.5 * (k[2] * P.Text[0] - k[0] * P.Text[2]),
                       -0.5 * (k[0] * P.Text[1] - k[1] * P.Text[0])};  // Q^T k
        const double a_ = P.axes[0], b_ = P.axes[1];
        const double e2 = a_ > b_ && b_ == P.axes[2] ? 1.0 - (b_ / a_) * (b_ / a_) : 0.0;
        double xk = sqrt(k2) * eq_radius(P);
        if (e2 >= E_LINE * E_LINE) {
            const double p[3] = {Rm[0][0], Rm[1][0], Rm[2][0]};
            const double Tp = P.Text[0] * p[0] + P.Text[1] * p[1] + P.Text[2] * p[2];
            const double Tc[3] = {P.Text[0] - Tp * p[0], P.Text[1] - Tp * p[1], P.Text[2] - Tp * p[2]};
            const double m[3] = {Tc[1] * p[2] - Tc[2] * p[1], Tc[2] * p[0] - Tc[0] * p[2], Tc[0] * p[1] - Tc[1] * p[0]};
            const double cs = 0.5 * e2 / (2.0 - e2);
            const double km = k[0] * m[0] + k[1] * m[1] + k[2] * m[2], kp = k[0] * p[0] + k[1] * p[1] + k[2] * p[2];
            for (int j = 0; j < 3; ++j) g[j] += cs * (km * p[j] + kp * m[j]);
            xk = xa;
        }
        const double j1k = (sin(xk) - xk * cos(xk)) / (xk * xk * xk);  // j1(kappa) / kappa
        const double kg = k[0] * g[0] + k[1] * g[1] + k[2] * g[2];
        double sp, cp;
        sincos(-(k[0] * P.xc[0] + k[1] * P.xc[1] + k[2] * P.xc[2]), &sp, &cp);  // exp(-i k . x_c)
        for (int a = 0; a < 3; ++a) {
            // u_hat / V = (I - k k / k^2) f_hat / (mu k^2 V), f_hat = F sinc - 3 i g j1k
            const double re = (P.Fext[a] - k[a] * kF / k2) * sinc / (mu * k2) / V;
            const double im = -3.0 * (g[a] - k[a] * kg / k2) * j1k / (mu * k2) / V;
            c[2 * a] += re * cp - im * sp;
            c[2 * a + 1] += re * sp + im * cp;
        }
        // p_hat / V = -i (k . f_hat) / (k^2 V) = pre + i pim
        const double pre = -3.0 * kg * j1k / k2 / V, pim = -kF * sinc / k2 / V;
        c[6] += pre * cp - pim * sp;
        c[7] += pre * sp + pim * cp;
    }
    for (int a = 0; a < UF; ++a) {
        c[2 * a] -= S[(long long)id * MC + 2 * a] / V;
        c[2 * a + 1] -= S[(long long)id * MC + 2 * a + 1] / V;
    }
}

// partial sums over the fluid nodes of each tile: sum of u (3), of p u (3),
// of p and the count
__global__ __launch_bounds__(TILE) void k_stokes_sum(const BoxDesc* __restrict__ boxes,
                                                     const int* __restrict__ tile_box,
                                                     const uint16_t* __restrict__ omap,
                                                     const PartDev* __restrict__ parts,
                                                     const double* __restrict__ uf, long long base, int only_box,
                                                     const double* __restrict__ coef,
                                                     double* __restrict__ partial) {
    __shared__ double red[NPART][TILE];
    __shared__ RowCoefs rc;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int bi = tile_box[tile];
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + tid;
    double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool started = only_box < 0 || bi == only_box;  // uniform over the block
    if (started) row_coefs(B, coef + (long long)bi * WM * MC, (tile - B.tile0) * TILE, rc);
    if (started && s < B.n && omap[B.ooff + s] == 0) {
        const int x = s % B.nx, t = s / B.nx, y = t % B.ny, z = t / B.ny;
        double u[UF];
        start_velocity(B, 0, parts, uf, base, rc, s, x, y, z, u);
        for (int k = 0; k < 3; ++k) {
            v[k] = u[k];
            v[3 + k] = u[3] * u[k];
        }
        v[6] = u[3];
        v[7] = 1.0;
    }
    for (int k = 0; k < NPART; ++k) red[k][tid] = v[k];
    __syncthreads();
    for (int h = TILE / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int k = 0; k < NPART; ++k) red[k][tid] += red[k][tid + h];
        __syncthreads();
    }
    if (tid < NPART) partial[(long long)tile * NPART + tid] = red[tid][0];
}

// One wave per box: the mean pressure pbar of its fluid nodes and the
// uniform velocity ubar removed from them.  A fluid node gets the density
// rho = rho0 + 3 (p - pbar) (p = c_s^2 (rho - rho0)), so the fluid's mass is
// unchanged, and ubar = (sum rho u + sum_p M U) / (N rho0) makes the box's
// momentum sum rho (u - ubar) + sum_p M U zero.
__global__ __launch_bounds__(64) void k_stokes_mean(const BoxDesc* __restrict__ boxes,
                                                    const PartDev* __restrict__ parts, int np,
                                                    const double* __restrict__ partial, double rho0,
                                                    double* __restrict__ ubar) {
    const int b = blockIdx.x, lane = threadIdx.x;  // one 64-wide work-group per box
    const BoxDesc& B = boxes[b];
    double S[NPART] = {0, 0, 0, 0, 0, 0, 0, 0}, MU[3] = {0, 0, 0};
    for (int t = B.tile0 + lane; t < B.tile0 + B.ntiles; t += 64)
        for (int k = 0; k < NPART; ++k) S[k] += partial[(long long)t * NPART + k];
    for (int p = lane; p < np; p += 64)
        if (parts[p].box == b)
            for (int k = 0; k < 3; ++k) MU[k] += parts[p].M * parts[p].U[k];
    for (int k = 0; k < NPART; ++k) S[k] = wave_sum(S[k]);
    for (int k = 0; k < 3; ++k) MU[k] = wave_sum(MU[k]);
    if (lane != 0) return;
    const double N = S[7], pbar = N > 0 ? S[6] / N : 0.0;
    double J[3];
    for (int k = 0; k < 3; ++k) J[k] = rho0 * S[k] + 3.0 * (S[3 + k] - pbar * S[k]) + MU[k];
    for (int k = 0; k < 3; ++k) ubar[4 * b + k] = N > 0 ? J[k] / (N * rho0) : 0.0;
    ubar[4 * b + 3] = pbar;
}

template <int ST, int Q>
__global__ __launch_bounds__(TILE) void k_stokes_write(const BoxDesc* __restrict__ boxes,
                                                       const int* __restrict__ tile_box,
                                                       const uint16_t* __restrict__ omap,
                                                       const PartDev* __restrict__ parts,
                                                       const double* __restrict__ uf, long long base,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ ubar,
                                                       typename Store<ST>::T* __restrict__ f, KParams kp,
                                                       int only_box) {
    using S = Store<ST>;
    __shared__ RowCoefs rc;
    const int tile = blockIdx.x;
    const int bi = tile_box[tile];
    if (only_box >= 0 && bi != only_box) return;  // uniform over the block
    const BoxDesc& B = boxes[bi];
    row_coefs(B, coef + (long long)bi * WM * MC, (tile - B.tile0) * TILE, rc);
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    const uint16_t owner = omap[B.ooff + s];
    if (owner == 0xFFFF) return;
    const int nx = B.nx, ny = B.ny, nz = B.nz;
    const int x = s % nx, t = s / nx, y = t % ny, z = t / ny;
    double u[UF];
    start_velocity(B, owner, parts, uf, base, rc, s, x, y, z, u);
    const double rho0 = kp.rho0;
    double rho = rho0;
    if (owner == 0) {
        for (int k = 0; k < 3; ++k) u[k] -= ubar[4 * bi + k];
        rho = rho0 + 3.0 * (u[3] - ubar[4 * bi + 3]);
    }
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    typename S::T* fb = f + B.foff;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double dev = wgt<Q>(i) * ((rho - rho0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        // the slot node (x, y, z) reads f_i from at the next step (no walls here)
        int d, slot;
        pre_slot_open(kp.conv, i, x, y, z, nx, ny, nz, d, slot);
        S::st64(fb + (long long)d * B.stride + slot, dev, kp.scale);
    }
}

// ---------------------------------------------------------------------------
// Fallback monitor of warm-started boxes, one work-group per box, run every
// monitor period.  W0, the viscous time 2 a^2 / nu of the box's largest
// particle (a its largest semi-axis), is the time in which a particle sheds
// the error of its start.  The first check at least Wref = W0 / 4 steps after
// the warm start takes the reference: the flow energy E = sum |j|^2 over the
// box's fluid and every particle's V = (U, a Omega).  The first check at
// least W0 steps after it decides from the residuals (the relative changes
// since the reference: |E - E_ref| / (2 E), E being quadratic in the velocity,
// and the largest |V - V_ref| / |V| over the box's particles) and the
// prediction.  The box misses when more than a quarter of its particles
// (MON_MISS_SHARE) are further than tol from their predictions: a lone
// particle on its own miss, while in a crowded box the interactions can
// carry a few particles away from any one-particle prediction without the
// start being wrong.
//   no miss   accepted;
//   a miss while a residual exceeds tol (the run moves away from the
//     prediction)   fallback: the box restarts from the plain start (fluid and
//     particles at rest, pending transition book-keeping dropped), its steps
//     so far spent;
//   a miss with both residuals below tol (the run has settled elsewhere)
//     kept, its sample to be added to the training data.
constexpr double MON_MISS_SHARE = 0.25;
__global__ __launch_bounds__(256) void k_warm_monitor(const BoxDesc* __restrict__ boxes, BoxMon* __restrict__ mon,
                                                      const double* __restrict__ partial, PartDev* __restrict__ parts,
                                                      int np, const double* __restrict__ pred,
                                                      double* __restrict__ vref, long long step) {
    const int b = blockIdx.x, tid = threadIdx.x;
    BoxMon& M = mon[b];
    __shared__ double red[4][4];
    __shared__ int phase;  // 0 nothing, 1 take the reference, 2 decide
    __shared__ int decide;
    if (M.status != MON_PENDING) {
        if (tid == 0) M.reset = 0;
        return;
    }
    if (tid == 0) {
        const long long age = step - M.t0;
        phase = M.t_ref < 0 ? (age >= M.Wref ? 1 : 0) : (age >= M.W0 && step > M.t_ref ? 2 : 0);
        M.reset = 0;
    }
    __syncthreads();
    if (phase == 0) return;  // uniform over the block
    const BoxDesc& B = boxes[b];
    // the box's flow energy, tile partials summed in a fixed order
    double e = 0.0;
    for (int t = B.tile0 + tid; t < B.tile0 + B.ntiles; t += blockDim.x) e += partial[t];
    // the box's particles: the largest relative change since the reference,
    // and how many of them miss their prediction
    double dv = 0.0, miss = 0.0, cnt = 0.0;
    for (int p = tid; p < np; p += blockDim.x) {
        const PartDev& P = parts[p];
        if (P.box != b) continue;
        const double a = fmax(P.axes[0], fmax(P.axes[1], P.axes[2]));
        const double V[6] = {P.U[0], P.U[1], P.U[2], a * P.W[0], a * P.W[1], a * P.W[2]};
        double* vr = vref + 6 * (long long)p;
        const double* pr = pred + 6 * (long long)p;
        if (phase == 1) {
            for (int k = 0; k < 6; ++k) vr[k] = V[k];
            continue;
        }
        double d2 = 0, v2 = 0, m2 = 0, p2 = 0;
        for (int k = 0; k < 6; ++k) {
            const double pk = k < 3 ? pr[k] : a * pr[k];
            d2 += (V[k] - vr[k]) * (V[k] - vr[k]);
            v2 += V[k] * V[k];
            m2 += (V[k] - pk) * (V[k] - pk);
            p2 += pk * pk;
        }
        dv = fmax(dv, v2 > 0 ? sqrt(d2 / v2) : 0.0);
        if (m2 > M.tol * M.tol * p2) miss += 1.0;
        cnt += 1.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o);
        dv = fmax(dv, __shfl_xor(dv, o));
        miss += __shfl_xor(miss, o);
        cnt += __shfl_xor(cnt, o);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = e;
        red[1][tid >> 6] = dv;
        red[2][tid >> 6] = miss;
        red[3][tid >> 6] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0, DV = 0, MISS = 0, N = 0;
        for (int k = 0; k < 4; ++k) {
            E += red[0][k];
            DV = fmax(DV, red[1][k]);
            MISS += red[2][k];
            N += red[3][k];
        }
        int dec = 0;
        if (phase == 1) {
            M.E_ref = E;
            M.t_ref = step;
        } else {
            M.res_flow = E > 0 ? 0.5 * fabs(E - M.E_ref) / E : 0.0;
            M.res_part = DV;
            const bool conv = M.res_flow < M.tol && M.res_part < M.tol;
            dec = MISS <= MON_MISS_SHARE * N ? MON_ACCEPTED : (conv ? MON_STEADY_MISS : MON_FALLBACK);
            M.status = dec;
            M.t_decided = step;
        }
        M.reset = dec == MON_FALLBACK ? 1 : 0;
        decide = dec;
    }
    __syncthreads();
    if (decide != MON_FALLBACK) return;
    for (int p = tid; p < np; p += blockDim.x) {  // the box's particles to rest
        PartDev& P = parts[p];
        if (P.box != b) continue;
        for (int k = 0; k < 3; ++k) {
            P.U[k] = P.W[k] = 0.0;
            P.Pp[k] = P.Lp[k] = 0.0;
        }
        P.dm = 0.0;
    }
}

// Every population slot of a box whose check fell back is set to rest
// (deviation 0 in every storage format and layout).
template <typename T>
__global__ __launch_bounds__(TILE) void k_box_reset(const BoxDesc* __restrict__ boxes, const int* __restrict__ tile_box,
                                                    const BoxMon* __restrict__ mon, T* __restrict__ f, int q) {
    const int tile = blockIdx.x;
    const int bi = tile_box[tile];
    if (!mon[bi].reset) return;
    const BoxDesc& B = boxes[bi];
    const int s = (tile - B.tile0) * TILE + (int)threadIdx.x;
    if (s >= B.n) return;
    for (int i = 0; i < q; ++i) f[B.foff + (long long)i * B.stride + s] = T(0);
}

hipError_t launch_warm_monitor(const BoxDesc* boxes, int nboxes, const int* tile_box, int ntiles, BoxMon* mon,
                               const double* partial, PartDev* parts, int np, const double* pred, double* vref,
                               long long step, void* f, int storage, int q, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_monitor, dim3(nboxes), dim3(256), 0, st, boxes, mon, partial, parts, np, pred, vref,
                       step);
    const int es = storage_bytes(storage);
    if (es == 8)
        hipLaunchKernelGGL((k_box_reset<unsigned long long>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, mon,
                           (unsigned long long*)f, q);
    else if (es == 4)
        hipLaunchKernelGGL((k_box_reset<uint32_t>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, mon,
                           (uint32_t*)f, q);
    else
        hipLaunchKernelGGL((k_box_reset<uint16_t>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, mon,
                           (uint16_t*)f, q);
    return hipGetLastError();
}

hipError_t launch_warm_features(const BoxDesc* boxes, const PartDev* parts, int np, double mu, float* X, double* s,
                                hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_features, dim3((np + 63) / 64), dim3(64), 0, st, boxes, parts, np, mu, X, s);
    return hipGetLastError();
}

hipError_t launch_warm_apply(PartDev* parts, int np, const float* Y, const double* s, double mu, double* pred,
                             int only_box, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_apply, dim3((np + 63) / 64), dim3(64), 0, st, parts, np, Y, s, mu, pred, only_box);
    return hipGetLastError();
}

hipError_t launch_warm_targets(const PartDev* parts, int np, const double* s, double mu, float* Y, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_targets, dim3((np + 63) / 64), dim3(64), 0, st, parts, np, s, mu, Y);
    return hipGetLastError();
}

size_t stokes_scratch_doubles(int nboxes, int ntiles) {
    return (size_t)nboxes * WM * MC * 2 + (size_t)ntiles * NPART + 4 * (size_t)nboxes;
}
int stokes_free_doubles() { return UF; }

hipError_t launch_stokes_start(const BoxDesc* boxes, int nboxes, const int* tile_box, int ntiles,
                               const uint16_t* omap, const PartDev* parts, int np, double mu, double* scratch,
                               double* uf, long long base, void* f, const KParams& kp, int only_box, hipStream_t st) {
    double* S = scratch;
    double* C = S + (size_t)nboxes * WM * MC;
    double* partial = C + (size_t)nboxes * WM * MC;
    double* ubar = partial + (size_t)ntiles * NPART;
    hipLaunchKernelGGL(k_stokes_free, dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, parts, np, mu, only_box, base,
                       uf);
    hipLaunchKernelGGL(k_stokes_modes, dim3((2 * WK + 1) * (2 * WK + 1) * nboxes), dim3(256), 0, st, boxes, uf, base,
                       only_box, S);
    hipLaunchKernelGGL(k_stokes_coef, dim3((nboxes * WM + 127) / 128), dim3(128), 0, st, boxes, nboxes, parts, np, mu,
                       S, C);
    hipLaunchKernelGGL(k_stokes_sum, dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box, omap, parts, uf, base,
                       only_box, C, partial);
    hipLaunchKernelGGL(k_stokes_mean, dim3(nboxes), dim3(64), 0, st, boxes, parts, np, partial, kp.rho0, ubar);
    auto write = [&](auto q) {
        constexpr int Q = decltype(q)::value;
        switch (kp.storage) {
            case ST_F64:
                hipLaunchKernelGGL((k_stokes_write<ST_F64, Q>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                                   omap, parts, uf, base, C, ubar, (double*)f, kp, only_box);
                break;
            case ST_F32:
                hipLaunchKernelGGL((k_stokes_write<ST_F32, Q>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                                   omap, parts, uf, base, C, ubar, (float*)f, kp, only_box);
                break;
            case ST_F16:
                hipLaunchKernelGGL((k_stokes_write<ST_F16, Q>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                                   omap, parts, uf, base, C, ubar, (typename Store<ST_F16>::T*)f, kp, only_box);
                break;
            default:
                hipLaunchKernelGGL((k_stokes_write<ST_BF16, Q>), dim3(ntiles), dim3(TILE), 0, st, boxes, tile_box,
                                   omap, parts, uf, base, C, ubar, (typename Store<ST_BF16>::T*)f, kp, only_box);
        }
    };
    if (kp.q == 27) write(std::integral_constant<int, 27>{});
    else write(std::integral_constant<int, 19>{});
    return hipGetLastError();
}

}  // namespace lbd
