/*
 * lbe_oracle.c - FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see lbe_oracle.h).
 *
 * Follows the paper (arXiv 2403.05443) step by step:
 *   Sec. II.A      lattice, moments, equilibrium, collision, streaming
 *   Sec. II.B      ellipsoid surface, boundary links, bounce-back, eqs. fb, ub
 *   Sec. II.C      eqs. Fsplit..Tdiscrete (implicit solve), posupdate,
 *                  qevolution, qnplus0/qnplus1
 *   Sec. II.D      body inertia, eq. vectrotn, eq. Irot, eq. Irotdiff
 *   Sec. III.D     squirmer slip, eqs. squirmer, ubsquirmer
 *   Appendix A     order of the ten steps of one iteration
 * Readings where the paper is silent or ambiguous:
 *   R1  the collision sign of Sec. II.A is taken as f* = f - (f - f_eq)/tau;
 *   R2  D3Q19 velocities/weights are the textbook set; order as in lbell.h;
 *   R3  nodes at integer coordinates; solid iff Q < 1 (strict); minimum image;
 *   R4  body x axis carries semi-axis a (I1 = M(b^2+c^2)/5 is about it);
 *   R5  quaternion: Hamilton, scalar first, body->lab, Omega in lab frame;
 *   R6  dI/dt uses Omega(t) (step 4 precedes the solve);
 *   R7  bounce-back uses U(t+1), Omega(t+1) and x_c(t) (step 6 precedes 7);
 *   R8  external force/torque enter the right-hand side of the solve;
 *   R9  a node that changes side carries the rest density rho0 with it (no
 *       fluid inside the particle, Sec. II.B): a covered node's momentum and
 *       its mass in excess of rho0 go to the particle; an uncovered node gets
 *       f = f_eq(rho0, U + Omega x r), its momentum paid by the particle; the
 *       excess mass dm is returned at the next bounce-back spread over the
 *       links as dm * w_b / sum_b w_b.  Conserved: the box mass counting
 *       every particle node at rho0 (or_get_mass);
 *   R10 optional counter-force: a uniform force density g = -sum F_ext / N on
 *       all matter of the box (N = non-wall nodes), so total momentum stays
 *       zero: every fluid node gets f* += w_i (c_i . g)/c_s^2 after collision
 *       and every particle gets (its solid node count) * g on top of F_ext;
 *   R11 squirmer slip evaluated at the boundary node with the axial
 *       coordinate clamped to [-a, a];
 *   R12 the Couette start includes the first-order non-equilibrium part.
 */
#include "lbe_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NQMAX 27
#define CS2 (1.0 / 3.0)

/* Sec. II.A: velocity sets (textbook, reading R2).  D3Q19: rest, the six
   axis vectors, the twelve edge vectors; D3Q27 adds the eight corner
   vectors (appended, each followed by its opposite). */
static const int CX[NQMAX] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                              1, -1, 1, -1, 1, -1, -1, 1};
static const int CY[NQMAX] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                              1, -1, 1, -1, -1, 1, 1, -1};
static const int CZ[NQMAX] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                              1, -1, -1, 1, 1, -1, 1, -1};
/* weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216 */
static const double WT19[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                1.0 / 36};
static const double WT27[27] = {8.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,
                                2.0 / 27,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
                                1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
                                1.0 / 54,  1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216,
                                1.0 / 216, 1.0 / 216, 1.0 / 216};

static const double* weights_of(int lattice) { return lattice == 27 ? WT27 : WT19; }

/* index of -c_i, found once by search over the velocity table (the D3Q19
   part of the table is closed under negation, so one table serves both) */
static int opposite_search(int i) {
    int j;
    for (j = 0; j < NQMAX; j++)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

static int OPPT[NQMAX];
static int opp_ready = 0;
static int opposite(int i) {
    if (!opp_ready) {
        int j;
        for (j = 0; j < NQMAX; j++) OPPT[j] = opposite_search(j);
        opp_ready = 1;
    }
    return OPPT[i];
}


typedef struct {
    double xc[3], xu[3], q[4], U[3], W[3];
    double axes[3], ia2[3], M, Ib[3];
    double Fext[3], Text[3], B1, B2;
    double zeta[36];          /* rows: F (3), T (3); cols: U (3), Omega (3) */
    double dm, Pp[3], Lp[3];  /* pending transition book-keeping (R9)       */
    double F[3], T[3];        /* hydrodynamic force / torque of last step   */
    double wsum;              /* sum of w_b over the links                  */
    double qprev[4];          /* orientation one step before (finite-difference dI/dt) */
    int nlinks, lcap;
    int* lsite;
    int* ldir;
} opart;

struct or_sim {
    int nx, ny, nz, n;
    int q;              /* lattice: 19 or 27 velocities */
    const double* wt;   /* its weights                  */
    int coll;
    double tau, taum, rho0;
    int walls;
    double ulo[3], uhi[3];
    int counterforce;
    int rotation;        /* 0 eq. Irotdiff with I(t); 1 finite-difference dI/dt;
                            2 predictor-corrector for I(t + dt) (reading R21) */
    double* f;   /* pre-collision f[site*q+i], meaningful on fluid nodes */
    double* fs;  /* post-collision                                       */
    int* node;   /* 0 fluid, p+1 solid of particle p, -1 wall            */
    int np, pcap;
    opart* p;
    long long step;
    int overlaps;
};

static int site_of(const or_sim* s, int x, int y, int z) { return x + s->nx * (y + s->ny * z); }
static int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

/* minimum-image separation (reading R3) */
static double minimg(double d, int n) {
    if (d >= 0.5 * n) d -= n;
    else if (d < -0.5 * n) d += n;
    return d;
}

static void cross(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

/* ---------------- Sec. II.A: equilibrium and collision ------------------- */

static void equilibrium(int q, const double* wt, double rho, const double u[3], double* feq) {
    int i;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (i = 0; i < q; i++) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = rho * wt[i] * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

void or_equilibrium(double rho, const double u[3], double feq[19]) { equilibrium(19, WT19, rho, u, feq); }

void or_equilibrium_q(int lattice, double rho, const double u[3], double* feq) {
    equilibrium(lattice, weights_of(lattice), rho, u, feq);
}

static void moments(int q, const double* f, double* rho, double u[3]) {
    int i;
    double r = 0, j[3] = {0, 0, 0};
    for (i = 0; i < q; i++) {
        r += f[i];
        j[0] += f[i] * CX[i];
        j[1] += f[i] * CY[i];
        j[2] += f[i] * CZ[i];
    }
    *rho = r;
    u[0] = j[0] / r;
    u[1] = j[1] / r;
    u[2] = j[2] / r;
}

void or_collide_node(const or_sim* s, const double* f, double* out) {
    double rho, u[3], feq[NQMAX];
    int i;
    moments(s->q, f, &rho, u);
    equilibrium(s->q, s->wt, rho, u, feq);
    if (s->coll == 0) {
        /* BGK, reading R1 */
        for (i = 0; i < s->q; i++) out[i] = f[i] - (f[i] - feq[i]) / s->tau;
    } else if (s->coll == 1) {
        /* two-relaxation-time: symmetric part with tau+, antisymmetric with tau- */
        for (i = 0; i < s->q; i++) {
            int o = opposite(i);
            double fp = 0.5 * (f[i] + f[o]), fm = 0.5 * (f[i] - f[o]);
            double ep = 0.5 * (feq[i] + feq[o]), em = 0.5 * (feq[i] - feq[o]);
            out[i] = f[i] - (fp - ep) / s->tau - (fm - em) / s->taum;
        }
    } else {
        /* hydrodynamic modes (rho, j, second moments) kept / relaxed with tau,
           ghost modes set to equilibrium (zero): Hermite reconstruction */
        double P[3][3] = {{0}}, Pneq[3][3], c[3];
        int a, b;
        for (i = 0; i < s->q; i++) {
            c[0] = CX[i]; c[1] = CY[i]; c[2] = CZ[i];
            for (a = 0; a < 3; a++)
                for (b = 0; b < 3; b++) P[a][b] += f[i] * c[a] * c[b];
        }
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++)
                Pneq[a][b] = P[a][b] - rho * CS2 * (a == b) - rho * u[a] * u[b];
        for (i = 0; i < s->q; i++) {
            double cu, qp = 0;
            c[0] = CX[i]; c[1] = CY[i]; c[2] = CZ[i];
            cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
            for (a = 0; a < 3; a++)
                for (b = 0; b < 3; b++) {
                    double Qab = c[a] * c[b] - CS2 * (a == b);
                    qp += Qab * (rho * u[a] * u[b] + (1.0 - 1.0 / s->tau) * Pneq[a][b]);
                }
            out[i] = s->wt[i] * (rho + rho * cu / CS2 + qp / (2.0 * CS2 * CS2));
        }
    }
}

/* -------------- Sec. II.B: ellipsoid surface, eq. ellipsoidsurface -------- */

/* eq. vectrotn with q^-1: body-frame coordinates of a lab vector.  The
   expression order is fixed and FP contraction is off, because solid/fluid
   decisions are compared bit for bit with the GPU library, which evaluates
   the same expression in the same order. */
static void to_body(const double q[4], const double d[3], double o[3]) {
    double q0 = q[0], p1 = -q[1], p2 = -q[2], p3 = -q[3];
    double a0 = (2.0 * q0) * q0 - 1.0;
    double ps = (p1 * d[0] + p2 * d[1]) + p3 * d[2];
    double cx = p2 * d[2] - p3 * d[1];
    double cy = p3 * d[0] - p1 * d[2];
    double cz = p1 * d[1] - p2 * d[0];
    o[0] = (a0 * d[0] + (2.0 * ps) * p1) + (2.0 * q0) * cx;
    o[1] = (a0 * d[1] + (2.0 * ps) * p2) + (2.0 * q0) * cy;
    o[2] = (a0 * d[2] + (2.0 * ps) * p3) + (2.0 * q0) * cz;
}

static int inside_ia2(int nx, int ny, int nz, const double xc[3], const double ia2[3],
                      const double q[4], int x, int y, int z) {
    double d[3], b[3], Q;
    d[0] = minimg((double)x - xc[0], nx);
    d[1] = minimg((double)y - xc[1], ny);
    d[2] = minimg((double)z - xc[2], nz);
    to_body(q, d, b);
    Q = ((b[0] * b[0]) * ia2[0] + (b[1] * b[1]) * ia2[1]) + (b[2] * b[2]) * ia2[2];
    return Q < 1.0;
}

int or_inside(int nx, int ny, int nz, const double xc[3], const double axes[3],
              const double q[4], int x, int y, int z) {
    double ia2[3];
    int k;
    for (k = 0; k < 3; k++) ia2[k] = 1.0 / (axes[k] * axes[k]);
    return inside_ia2(nx, ny, nz, xc, ia2, q, x, y, z);
}

/* -------------- quaternion algebra (Sec. II.C, II.D) --------------------- */

static void qmul(const double a[4], const double b[4], double r[4]) {
    double t[4];
    t[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    t[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    t[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    t[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    memcpy(r, t, sizeof t);
}

/* each column of the 4x4 matrix X is a quaternion; Y[:,k] = a X[:,k] b */
static void sandwich_cols(const double a[4], const double X[4][4], const double b[4],
                          double Y[4][4]) {
    int k, r;
    for (k = 0; k < 4; k++) {
        double col[4], t[4];
        for (r = 0; r < 4; r++) col[r] = X[r][k];
        qmul(a, col, t);
        qmul(t, b, t);
        for (r = 0; r < 4; r++) Y[r][k] = t[r];
    }
}

static void transpose4(const double X[4][4], double Y[4][4]) {
    int r, c;
    double t[4][4];
    for (r = 0; r < 4; r++)
        for (c = 0; c < 4; c++) t[c][r] = X[r][c];
    memcpy(Y, t, sizeof t);
}

/* ( a ( b I c )^T d )^T with I the 4x4 pure-quaternion inertia tensor */
static void irot_term(const double a[4], const double b[4], const double c[4],
                      const double d[4], const double I4[4][4], double out[4][4]) {
    double Y[4][4];
    sandwich_cols(b, I4, c, Y);
    transpose4(Y, Y);
    sandwich_cols(a, Y, d, Y);
    transpose4(Y, out);
}

static void inertia4(const double Ib[3], double I4[4][4]) {
    memset(I4, 0, 16 * sizeof(double));
    I4[1][1] = Ib[0];
    I4[2][2] = Ib[1];
    I4[3][3] = Ib[2];
}

/* eq. Irot: I' = ( q ( q I q^-1 )^T q^-1 )^T */
void or_inertia_lab(const double q[4], const double Ib[3], double out[9]) {
    double I4[4][4], R[4][4], qi[4] = {q[0], -q[1], -q[2], -q[3]};
    int r, c;
    inertia4(Ib, I4);
    irot_term(q, q, qi, qi, I4, R);
    for (r = 0; r < 3; r++)
        for (c = 0; c < 3; c++) out[3 * r + c] = R[r + 1][c + 1];
}

/* eq. Irotdiff with qdot from eq. qevolution: four product-rule terms */
void or_inertia_dot(const double q[4], const double Ib[3], const double W[3], double out[9]) {
    double I4[4][4], T[4][4], S[4][4] = {{0}};
    double qi[4] = {q[0], -q[1], -q[2], -q[3]};
    double Wq[4] = {0.0, W[0], W[1], W[2]}, qd[4], qdi[4];
    int r, c, k;
    qmul(Wq, q, qd);
    for (k = 0; k < 4; k++) qd[k] *= 0.5;
    qdi[0] = qd[0]; qdi[1] = -qd[1]; qdi[2] = -qd[2]; qdi[3] = -qd[3];
    inertia4(Ib, I4);
    irot_term(qd, q, qi, qi, I4, T);
    for (r = 0; r < 4; r++) for (c = 0; c < 4; c++) S[r][c] += T[r][c];
    irot_term(q, qd, qi, qi, I4, T);
    for (r = 0; r < 4; r++) for (c = 0; c < 4; c++) S[r][c] += T[r][c];
    irot_term(q, q, qdi, qi, I4, T);
    for (r = 0; r < 4; r++) for (c = 0; c < 4; c++) S[r][c] += T[r][c];
    irot_term(q, q, qi, qdi, I4, T);
    for (r = 0; r < 4; r++) for (c = 0; c < 4; c++) S[r][c] += T[r][c];
    for (r = 0; r < 3; r++)
        for (c = 0; c < 3; c++) out[3 * r + c] = S[r + 1][c + 1];
}

/* eqs. qnplus0, qnplus1 */
void or_quat_update(const double q[4], const double Wm[3], double out[4]) {
    double nrm = sqrt(Wm[0] * Wm[0] + Wm[1] * Wm[1] + Wm[2] * Wm[2]);
    double qt[4];
    if (nrm == 0.0) {
        memcpy(out, q, 4 * sizeof(double));
        return;
    }
    qt[0] = cos(0.5 * nrm);
    qt[1] = sin(0.5 * nrm) * Wm[0] / nrm;
    qt[2] = sin(0.5 * nrm) * Wm[1] / nrm;
    qt[3] = sin(0.5 * nrm) * Wm[2] / nrm;
    qmul(qt, q, out);
}

/* Sec. II.C: "Gaussian elimination", with partial pivoting */
int or_solve6(const double A[36], const double b[6], double x[6]) {
    double M[6][7];
    int r, c, k;
    for (r = 0; r < 6; r++) {
        for (c = 0; c < 6; c++) M[r][c] = A[6 * r + c];
        M[r][6] = b[r];
    }
    for (k = 0; k < 6; k++) {
        int piv = k;
        for (r = k + 1; r < 6; r++)
            if (fabs(M[r][k]) > fabs(M[piv][k])) piv = r;
        if (!(fabs(M[piv][k]) > 1e-300)) return -1;
        if (piv != k)
            for (c = 0; c < 7; c++) {
                double t = M[k][c];
                M[k][c] = M[piv][c];
                M[piv][c] = t;
            }
        for (r = k + 1; r < 6; r++) {
            double m = M[r][k] / M[k][k];
            for (c = k; c < 7; c++) M[r][c] -= m * M[k][c];
        }
    }
    for (r = 5; r >= 0; r--) {
        double acc = M[r][6];
        for (c = r + 1; c < 6; c++) acc -= M[r][c] * x[c];
        x[r] = acc / M[r][r];
    }
    return 0;
}

/* Sec. III.D, eq. squirmer, reading R11.  d: boundary node minus centre (lab). */
void or_squirmer_slip(const double axes[3], const double q[4], double B1, double B2,
                      const double d[3], double us[3]) {
    double a = axes[0], bb = axes[1];
    double e[3], qe[4], t[4], xb[4] = {0, 1, 0, 0}, qi[4] = {q[0], -q[1], -q[2], -q[3]};
    double z, rv[3], r, ep[3], zc, eps, den, s[3], se, zeta;
    int k;
    /* e: body x axis in the lab frame, q (1,0,0) q^-1 */
    qmul(q, xb, t);
    qmul(t, qi, qe);
    e[0] = qe[1]; e[1] = qe[2]; e[2] = qe[3];
    z = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
    for (k = 0; k < 3; k++) rv[k] = d[k] - z * e[k];
    r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    us[0] = us[1] = us[2] = 0.0;
    if (r == 0.0) return;
    for (k = 0; k < 3; k++) ep[k] = rv[k] / r;
    zc = z > a ? a : (z < -a ? -a : z);
    eps = sqrt(1.0 - (bb * bb) / (a * a));
    den = sqrt(a * a - eps * eps * zc * zc);
    for (k = 0; k < 3; k++)
        s[k] = -sqrt(a * a - zc * zc) / den * e[k] + sqrt(1.0 - eps * eps) * zc / den * ep[k];
    se = s[0] * e[0] + s[1] * e[1] + s[2] * e[2];
    if (eps > 1e-8)
        zeta = (sqrt(r * r + (z + a * eps) * (z + a * eps)) -
                sqrt(r * r + (z - a * eps) * (z - a * eps))) / (2.0 * a * eps);
    else
        zeta = z / sqrt(r * r + z * z);
    for (k = 0; k < 3; k++) us[k] = -B1 * se * s[k] - B2 * zeta * se * s[k];
}

void or_lattice_q(int lattice, int* c, double* w) {
    int i;
    const double* wt = weights_of(lattice);
    for (i = 0; i < lattice; i++) {
        c[3 * i] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = wt[i];
    }
}

void or_lattice(int c[57], double w[19]) { or_lattice_q(19, c, w); }

/* ------------------------------- set-up ---------------------------------- */

static void init_fluid(or_sim* s, int init) {
    int x, y, z, i;
    for (z = 0; z < s->nz; z++)
        for (y = 0; y < s->ny; y++)
            for (x = 0; x < s->nx; x++) {
                int st = site_of(s, x, y, z);
                double u[3] = {0, 0, 0}, feq[NQMAX], g[3] = {0, 0, 0};
                if (s->walls && (y == 0 || y == s->ny - 1)) {
                    s->node[st] = -1;
                    for (i = 0; i < s->q; i++) s->f[st * s->q + i] = 0.0;
                    continue;
                }
                s->node[st] = 0;
                if (init == 1 && s->walls) {
                    /* linear profile between the half-way planes y=0.5, ny-1.5 */
                    double H = s->ny - 2.0;
                    int k;
                    for (k = 0; k < 3; k++) {
                        g[k] = (s->uhi[k] - s->ulo[k]) / H;
                        u[k] = s->ulo[k] + g[k] * (y - 0.5);
                    }
                }
                equilibrium(s->q, s->wt, s->rho0, u, feq);
                for (i = 0; i < s->q; i++) {
                    /* first-order Chapman-Enskog part: -tau w_i rho0 Q_i:grad u / c_s^2 */
                    double taus = s->tau;
                    double qg = CY[i] * (CX[i] * g[0] + CZ[i] * g[2]);
                    s->f[st * s->q + i] = feq[i] - taus * s->wt[i] * s->rho0 * qg / CS2;
                }
            }
}

or_sim* or_create_q(int nx, int ny, int nz, int collision, double tau, double magic,
                    int walls, const double ulo[3], const double uhi[3], int init,
                    int counterforce, int lattice) {
    or_sim* s;
    int k;
    if (lattice != 19 && lattice != 27) return NULL;
    s = (or_sim*)calloc(1, sizeof(or_sim));
    if (!s) return NULL;
    (void)opposite(0);
    s->q = lattice;
    s->wt = weights_of(lattice);
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->n = nx * ny * nz;
    s->coll = collision;
    s->tau = tau;
    s->taum = 0.5 + magic / (tau - 0.5);
    s->rho0 = 1.0;
    s->walls = walls;
    for (k = 0; k < 3; k++) {
        s->ulo[k] = ulo ? ulo[k] : 0.0;
        s->uhi[k] = uhi ? uhi[k] : 0.0;
    }
    s->counterforce = counterforce;
    s->f = (double*)calloc((size_t)s->n * s->q, sizeof(double));
    s->fs = (double*)calloc((size_t)s->n * s->q, sizeof(double));
    s->node = (int*)calloc((size_t)s->n, sizeof(int));
    s->pcap = 16;
    s->p = (opart*)calloc((size_t)s->pcap, sizeof(opart));
    init_fluid(s, init);
    return s;
}

or_sim* or_create(int nx, int ny, int nz, int collision, double tau, double magic,
                  int walls, const double ulo[3], const double uhi[3], int init,
                  int counterforce) {
    return or_create_q(nx, ny, nz, collision, tau, magic, walls, ulo, uhi, init, counterforce, 19);
}

int or_set_rotation(or_sim* s, int mode) {
    if (mode < 0 || mode > 2) return -1;
    s->rotation = mode;
    return 0;
}

void or_destroy(or_sim* s) {
    int k;
    if (!s) return;
    for (k = 0; k < s->np; k++) {
        free(s->p[k].lsite);
        free(s->p[k].ldir);
    }
    free(s->p);
    free(s->f);
    free(s->fs);
    free(s->node);
    free(s);
}

static double amax_of(const opart* p) {
    double m = p->axes[0];
    if (p->axes[1] > m) m = p->axes[1];
    if (p->axes[2] > m) m = p->axes[2];
    return m;
}

/* node r relative to the centre, minimum image */
static void rel(const or_sim* s, const double xc[3], double x, double y, double z, double r[3]) {
    r[0] = minimg(x - xc[0], s->nx);
    r[1] = minimg(y - xc[1], s->ny);
    r[2] = minimg(z - xc[2], s->nz);
}

/* eqs. drag1-drag4 over the current links of particle p, with x_c(t) */
static void build_links_and_zeta(or_sim* s, int pid) {
    opart* p = &s->p[pid];
    int b, a, dx, dy, dz, ext = (int)ceil(amax_of(p)) + 3;
    int x0 = (int)floor(p->xc[0]), y0 = (int)floor(p->xc[1]), z0 = (int)floor(p->xc[2]);
    int lo[3], len[3], n3[3] = {s->nx, s->ny, s->nz}, k;
    double K = 2.0 * s->rho0 / CS2;
    p->nlinks = 0;
    p->wsum = 0.0;
    /* scan a cube around the centre that holds the ellipsoid plus one node,
       clipped to the box so no node is visited twice; links in (site, b) order */
    lo[0] = x0 - ext; lo[1] = y0 - ext; lo[2] = z0 - ext;
    for (k = 0; k < 3; k++) {
        len[k] = 2 * ext + 2;
        if (len[k] >= n3[k]) {
            len[k] = n3[k];
            lo[k] = 0;
        }
    }
    for (dz = 0; dz < len[2]; dz++)
        for (dy = 0; dy < len[1]; dy++)
            for (dx = 0; dx < len[0]; dx++) {
                int x = ((lo[0] + dx) % s->nx + s->nx) % s->nx;
                int y = ((lo[1] + dy) % s->ny + s->ny) % s->ny;
                int z = ((lo[2] + dz) % s->nz + s->nz) % s->nz;
                int st = site_of(s, x, y, z);
                if (s->node[st] != 0) continue;
                for (b = 1; b < s->q; b++) {
                    int nb = site_of(s, wrapi(x + CX[b], s->nx), wrapi(y + CY[b], s->ny),
                                     wrapi(z + CZ[b], s->nz));
                    if (s->node[nb] != pid + 1) continue;
                    if (p->nlinks == p->lcap) {
                        p->lcap = p->lcap ? 2 * p->lcap : 1024;
                        p->lsite = (int*)realloc(p->lsite, sizeof(int) * p->lcap);
                        p->ldir = (int*)realloc(p->ldir, sizeof(int) * p->lcap);
                    }
                    p->lsite[p->nlinks] = st;
                    p->ldir[p->nlinks] = b;
                    p->nlinks++;
                }
            }
    memset(p->zeta, 0, sizeof p->zeta);
    for (a = 0; a < p->nlinks; a++) {
        int stl = p->lsite[a], bl = p->ldir[a];
        int x = stl % s->nx, y = (stl / s->nx) % s->ny, z = stl / (s->nx * s->ny);
        double cb[3] = {CX[bl], CY[bl], CZ[bl]}, r[3], rc[3];
        int i, j;
        rel(s, p->xc, x + 0.5 * cb[0], y + 0.5 * cb[1], z + 0.5 * cb[2], r);
        cross(r, cb, rc);
        p->wsum += s->wt[bl];
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) {
                p->zeta[6 * i + j] += K * s->wt[bl] * cb[i] * cb[j];               /* zeta_FU */
                p->zeta[6 * i + 3 + j] += K * s->wt[bl] * cb[i] * rc[j];           /* zeta_FW */
                p->zeta[6 * (3 + i) + j] += K * s->wt[bl] * rc[i] * cb[j];         /* zeta_TU */
                p->zeta[6 * (3 + i) + 3 + j] += K * s->wt[bl] * rc[i] * rc[j];     /* zeta_TW */
            }
    }
}

/* Appendix A step 8: remap nodes; returns the number of overlapping claims.
   apply = 0 at set-up (no transition book-keeping). */
static int remap(or_sim* s, int apply) {
    int* nn = (int*)malloc(sizeof(int) * (size_t)s->n);
    int st, pid, overl = 0;
    for (st = 0; st < s->n; st++) nn[st] = s->node[st] == -1 ? -1 : 0;
    for (pid = 0; pid < s->np; pid++) {
        opart* p = &s->p[pid];
        int ext = (int)ceil(amax_of(p)) + 2, dx, dy, dz;
        int x0 = (int)floor(p->xc[0]), y0 = (int)floor(p->xc[1]), z0 = (int)floor(p->xc[2]);
        for (dz = -ext; dz <= ext + 1; dz++)
            for (dy = -ext; dy <= ext + 1; dy++)
                for (dx = -ext; dx <= ext + 1; dx++) {
                    int x = wrapi(((x0 + dx) % s->nx + s->nx) % s->nx, s->nx);
                    int y = wrapi(((y0 + dy) % s->ny + s->ny) % s->ny, s->ny);
                    int z = wrapi(((z0 + dz) % s->nz + s->nz) % s->nz, s->nz);
                    int sn = site_of(s, x, y, z);
                    if (!inside_ia2(s->nx, s->ny, s->nz, p->xc, p->ia2, p->q, x, y, z)) continue;
                    if (nn[sn] == pid + 1) continue; /* window wrapped onto itself */
                    if (nn[sn] != 0) {
                        overl++;
                        continue; /* lower id (or the wall) keeps the node */
                    }
                    nn[sn] = pid + 1;
                }
    }
    if (apply) {
        for (st = 0; st < s->n; st++) {
            int o = s->node[st], m = nn[st], i;
            int x = st % s->nx, y = (st / s->nx) % s->ny, z = st / (s->nx * s->ny);
            if (o == m) continue;
            if (o > 0) {
                /* uncovered by particle o-1 (R9): f = f_eq(rho0, U + W x r) */
                opart* p = &s->p[o - 1];
                double r[3], wr[3], u[3], feq[NQMAX], L[3];
                rel(s, p->xc, x, y, z, r);
                cross(p->W, r, wr);
                for (i = 0; i < 3; i++) u[i] = p->U[i] + wr[i];
                equilibrium(s->q, s->wt, s->rho0, u, feq);
                for (i = 0; i < s->q; i++) s->f[st * s->q + i] = feq[i];  /* mass rho0: no excess */
                for (i = 0; i < 3; i++) u[i] *= s->rho0;
                cross(r, u, L);
                for (i = 0; i < 3; i++) {
                    p->Pp[i] -= u[i];
                    p->Lp[i] -= L[i];
                }
            }
            if (m > 0) {
                /* covered by particle m-1 (R9): momentum and excess mass to the particle */
                opart* p = &s->p[m - 1];
                double r[3], mass = 0, P[3] = {0, 0, 0}, L[3];
                for (i = 0; i < s->q; i++) {
                    double fi = s->f[st * s->q + i];
                    mass += fi;
                    P[0] += fi * CX[i];
                    P[1] += fi * CY[i];
                    P[2] += fi * CZ[i];
                }
                rel(s, p->xc, x, y, z, r);
                cross(r, P, L);
                p->dm += mass - s->rho0;
                for (i = 0; i < 3; i++) {
                    p->Pp[i] += P[i];
                    p->Lp[i] += L[i];
                }
            }
        }
    }
    memcpy(s->node, nn, sizeof(int) * (size_t)s->n);
    free(nn);
    for (pid = 0; pid < s->np; pid++) build_links_and_zeta(s, pid);
    return overl;
}

static void set_mass(opart* p, double rho_p) {
    double a = p->axes[0], b = p->axes[1], c = p->axes[2];
    p->M = rho_p * 4.0 / 3.0 * M_PI * a * b * c;
    /* Sec. II.D body-frame inertia */
    p->Ib[0] = p->M * (b * b + c * c) / 5.0;
    p->Ib[1] = p->M * (a * a + c * c) / 5.0;
    p->Ib[2] = p->M * (a * a + b * b) / 5.0;
}

int or_add_ellipsoid(or_sim* s, const double centre[3], const double axes[3], const double quat[4]) {
    opart* p;
    double nq;
    int k, ov, n3[3] = {s->nx, s->ny, s->nz};
    if (s->np == s->pcap) {
        s->pcap *= 2;
        s->p = (opart*)realloc(s->p, sizeof(opart) * (size_t)s->pcap);
    }
    p = &s->p[s->np];
    memset(p, 0, sizeof *p);
    nq = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    for (k = 0; k < 4; k++) p->q[k] = quat[k] / nq;
    for (k = 0; k < 4; k++) p->qprev[k] = p->q[k];
    for (k = 0; k < 3; k++) {
        double c = centre[k];
        if (c >= n3[k]) c -= n3[k] * floor(c / n3[k]);
        if (c < 0) c += n3[k] * ceil(-c / n3[k]);
        p->xc[k] = c;
        p->xu[k] = centre[k];
        p->axes[k] = axes[k];
        p->ia2[k] = 1.0 / (axes[k] * axes[k]);
    }
    set_mass(p, s->rho0);
    s->np++;
    ov = remap(s, 0);
    s->overlaps += ov;
    return ov ? -5 : s->np - 1;
}

int or_set_external(or_sim* s, int id, const double F[3], const double T[3]) {
    int k;
    if (id < 0 || id >= s->np) return -1;
    for (k = 0; k < 3; k++) {
        s->p[id].Fext[k] = F[k];
        s->p[id].Text[k] = T[k];
    }
    return 0;
}

int or_set_squirmer(or_sim* s, int id, double B1, double B2) {
    if (id < 0 || id >= s->np) return -1;
    s->p[id].B1 = B1;
    s->p[id].B2 = B2;
    return 0;
}

int or_set_velocity(or_sim* s, int id, const double U[3], const double W[3]) {
    int k;
    if (id < 0 || id >= s->np) return -1;
    for (k = 0; k < 3; k++) {
        s->p[id].U[k] = U[k];
        s->p[id].W[k] = W[k];
    }
    return 0;
}

int or_set_density(or_sim* s, int id, double rho_p) {
    if (id < 0 || id >= s->np) return -1;
    set_mass(&s->p[id], rho_p);
    return 0;
}

/* ------------------------ one iteration, Appendix A ---------------------- */

static int count_nonwall(const or_sim* s) {
    int st, n = 0;
    for (st = 0; st < s->n; st++) n += s->node[st] != -1;
    return n;
}

static int count_solid(const or_sim* s, int pid) {
    int st, n = 0;
    for (st = 0; st < s->n; st++) n += s->node[st] == pid + 1;
    return n;
}

static int step_once(or_sim* s) {
    const double K = 2.0 * s->rho0 / CS2;
    double g[3] = {0, 0, 0};
    int st, pid, k, rc = 0;

    if (s->counterforce && s->np > 0) {
        double Ft[3] = {0, 0, 0};
        int nall = count_nonwall(s);
        for (pid = 0; pid < s->np; pid++)
            for (k = 0; k < 3; k++) Ft[k] += s->p[pid].Fext[k];
        for (k = 0; k < 3; k++) g[k] = -Ft[k] / nall;
    }

    /* step 1: collision on every fluid node (+ counter-force, R10) */
#pragma omp parallel for schedule(static)
    for (st = 0; st < s->n; st++) {
        int i;
        if (s->node[st] != 0) continue;
        or_collide_node(s, &s->f[st * s->q], &s->fs[st * s->q]);
        for (i = 0; i < s->q; i++)
            s->fs[st * s->q + i] += s->wt[i] * s->rho0 * (CX[i] * g[0] + CY[i] * g[1] + CZ[i] * g[2]) / CS2;
    }

    /* step 2: streaming between fluid nodes; links into solid/wall nodes skipped */
#pragma omp parallel for schedule(static)
    for (st = 0; st < s->n; st++) {
        int x = st % s->nx, y = (st / s->nx) % s->ny, z = st / (s->nx * s->ny), i;
        if (s->node[st] != 0) continue;
        for (i = 0; i < s->q; i++) {
            int src = site_of(s, wrapi(x - CX[i], s->nx), wrapi(y - CY[i], s->ny),
                              wrapi(z - CZ[i], s->nz));
            if (s->node[src] == 0) s->f[st * s->q + i] = s->fs[src * s->q + i];
        }
    }

    for (pid = 0; pid < s->np; pid++) {
        opart* p = &s->p[pid];
        double F0[3] = {0, 0, 0}, T0[3] = {0, 0, 0}, Fs[3] = {0, 0, 0}, Ts[3] = {0, 0, 0};
        double Il[9], Id[9], A[36], rhs[6], sol[6], Iw[3], Fcf[3] = {0, 0, 0};
        int l, i, j;
        if (s->counterforce) {  /* R10: the counter-force density acting on the particle's nodes */
            int ns = count_solid(s, pid);
            for (k = 0; k < 3; k++) Fcf[k] = ns * g[k];
        }
        /* step 3: eqs. F0, T0 from post-collision populations (+ squirmer slip) */
        for (l = 0; l < p->nlinks; l++) {
            int stl = p->lsite[l], b = p->ldir[l];
            int x = stl % s->nx, y = (stl / s->nx) % s->ny, z = stl / (s->nx * s->ny);
            double cb[3] = {CX[b], CY[b], CZ[b]}, r[3], rc[3], fb = s->fs[stl * s->q + b];
            rel(s, p->xc, x + 0.5 * cb[0], y + 0.5 * cb[1], z + 0.5 * cb[2], r);
            cross(r, cb, rc);
            for (k = 0; k < 3; k++) {
                F0[k] += 2.0 * fb * cb[k];
                T0[k] += 2.0 * fb * rc[k];
            }
            if (p->B1 != 0.0 || p->B2 != 0.0) {
                double us[3], uc;
                or_squirmer_slip(p->axes, p->q, p->B1, p->B2, r, us);
                uc = us[0] * cb[0] + us[1] * cb[1] + us[2] * cb[2];
                for (k = 0; k < 3; k++) {
                    Fs[k] -= K * s->wt[b] * uc * cb[k];
                    Ts[k] -= K * s->wt[b] * uc * rc[k];
                }
            }
        }
        /* step 4: lab-frame inertia and its rate (eqs. Irot, Irotdiff), R6;
           or the finite difference (I(t) - I(t - dt)) / dt of Sec. II.D */
        or_inertia_lab(p->q, p->Ib, Il);
        if (s->rotation == 1) {
            double Ip[9];
            or_inertia_lab(p->qprev, p->Ib, Ip);
            for (k = 0; k < 9; k++) Id[k] = Il[k] - Ip[k];
        } else {
            or_inertia_dot(p->q, p->Ib, p->W, Id);
        }
        /* step 5: eqs. Fdiscrete, Tdiscrete (dt = 1) as one 6x6 system */
        for (i = 0; i < 6; i++)
            for (j = 0; j < 6; j++) A[6 * i + j] = p->zeta[6 * i + j];
        for (i = 0; i < 3; i++) {
            A[6 * i + i] += p->M;
            for (j = 0; j < 3; j++) A[6 * (3 + i) + 3 + j] += Il[3 * i + j] + Id[3 * i + j];
        }
        for (i = 0; i < 3; i++) Iw[i] = Il[3 * i] * p->W[0] + Il[3 * i + 1] * p->W[1] + Il[3 * i + 2] * p->W[2];
        for (i = 0; i < 3; i++) {
            rhs[i] = p->M * p->U[i] + F0[i] + Fs[i] + p->Fext[i] + Fcf[i] + p->Pp[i];
            rhs[3 + i] = Iw[i] + T0[i] + Ts[i] + p->Text[i] + p->Lp[i];
        }
        if (or_solve6(A, rhs, sol) != 0) return -6;
        if (s->rotation == 2) {
            /* R21: the solve above predicts Omega(t + dt); the orientation it
               gives (eqs. qnplus0/1 with the mean angular velocity) yields
               I(t + dt), and the rotational rows are solved again as the
               discrete balance I(t + dt) Omega(t + dt) - I(t) Omega(t) = dt T
               (the same right-hand side) */
            double Wm[3], qs[4], Is[9];
            for (i = 0; i < 3; i++) Wm[i] = 0.5 * (p->W[i] + sol[3 + i]);
            or_quat_update(p->q, Wm, qs);
            or_inertia_lab(qs, p->Ib, Is);
            for (i = 0; i < 3; i++)
                for (j = 0; j < 3; j++) A[6 * (3 + i) + 3 + j] = p->zeta[6 * (3 + i) + 3 + j] + Is[3 * i + j];
            if (or_solve6(A, rhs, sol) != 0) return -6;
        }
        for (i = 0; i < 3; i++) {
            double zf = 0, zt = 0;
            for (j = 0; j < 6; j++) {
                zf += p->zeta[6 * i + j] * sol[j];
                zt += p->zeta[6 * (3 + i) + j] * sol[j];
            }
            p->F[i] = F0[i] + Fs[i] + p->Pp[i] - zf;
            p->T[i] = T0[i] + Ts[i] + p->Lp[i] - zt;
            p->Pp[i] = 0.0;
            p->Lp[i] = 0.0;
        }
        /* keep U(t), Omega(t) for step 7 in sol's neighbours */
        {
            double Uold[3], Wold[3], r[3], Wm[3], qn[4];
            for (i = 0; i < 3; i++) {
                Uold[i] = p->U[i];
                Wold[i] = p->W[i];
                p->U[i] = sol[i];
                p->W[i] = sol[3 + i];
            }
            if (fabs(p->U[0]) > 0.5 || fabs(p->U[1]) > 0.5 || fabs(p->U[2]) > 0.5 ||
                !isfinite(p->U[0] + p->U[1] + p->U[2] + p->W[0] + p->W[1] + p->W[2]))
                rc = -6;
            /* step 6: bounce-back on the particle links (eqs. fb, ub, ubsquirmer), R7, R9 */
            for (l = 0; l < p->nlinks; l++) {
                int stl = p->lsite[l], b = p->ldir[l], bo = opposite(b);
                int x = stl % s->nx, y = (stl / s->nx) % s->ny, z = stl / (s->nx * s->ny);
                double cb[3] = {CX[b], CY[b], CZ[b]}, wr[3], ub[3], uc;
                rel(s, p->xc, x + 0.5 * cb[0], y + 0.5 * cb[1], z + 0.5 * cb[2], r);
                cross(p->W, r, wr);
                for (k = 0; k < 3; k++) ub[k] = p->U[k] + wr[k];
                if (p->B1 != 0.0 || p->B2 != 0.0) {
                    double us[3];
                    or_squirmer_slip(p->axes, p->q, p->B1, p->B2, r, us);
                    for (k = 0; k < 3; k++) ub[k] += us[k];
                }
                uc = ub[0] * cb[0] + ub[1] * cb[1] + ub[2] * cb[2];
                s->f[stl * s->q + bo] = s->fs[stl * s->q + b] - 2.0 * s->wt[b] * s->rho0 * uc / CS2 +
                                      (p->wsum > 0 ? p->dm * s->wt[b] / p->wsum : 0.0);
            }
            p->dm = 0.0;
            /* step 7: eq. posupdate and eqs. qnplus0/qnplus1 */
            for (i = 0; i < 3; i++) {
                int n3 = i == 0 ? s->nx : (i == 1 ? s->ny : s->nz);
                double dx = 0.5 * (p->U[i] + Uold[i]);
                p->xc[i] += dx;
                p->xu[i] += dx;
                if (p->xc[i] >= n3) p->xc[i] -= n3;
                if (p->xc[i] < 0.0) p->xc[i] += n3;
                Wm[i] = 0.5 * (Wold[i] + p->W[i]);
            }
            or_quat_update(p->q, Wm, qn);
            memcpy(p->qprev, p->q, sizeof qn);
            memcpy(p->q, qn, sizeof qn);
        }
    }

    /* step 6 for the walls: bounce-back with the wall velocity */
    if (s->walls) {
        for (st = 0; st < s->n; st++) {
            int x = st % s->nx, y = (st / s->nx) % s->ny, z = st / (s->nx * s->ny), b;
            if (s->node[st] != 0) continue;
            for (b = 1; b < s->q; b++) {
                int yy = y + CY[b];
                const double* uw;
                double uc;
                if (yy != 0 && yy != s->ny - 1) continue;
                (void)x; (void)z;
                uw = yy == 0 ? s->ulo : s->uhi;
                uc = uw[0] * CX[b] + uw[1] * CY[b] + uw[2] * CZ[b];
                s->f[st * s->q + opposite(b)] = s->fs[st * s->q + b] - 2.0 * s->wt[b] * s->rho0 * uc / CS2;
            }
        }
    }

    /* steps 8 and 9: remap with x_c(t+1), q(t+1); links and drag matrices */
    s->overlaps += remap(s, 1);
    s->step++;
    return rc;
}

int or_step(or_sim* s, int n) {
    int k, rc = 0;
    for (k = 0; k < n; k++) {
        int r = step_once(s);
        if (r != 0 && rc == 0) rc = r;
        if (r == -6) return r;
    }
    return rc;
}

/* ------------------------------- read-back -------------------------------- */

int or_get_particle(const or_sim* s, int id, double x[3], double q[4], double U[3], double W[3]) {
    const opart* p;
    if (id < 0 || id >= s->np) return -1;
    p = &s->p[id];
    if (x) memcpy(x, p->xu, 3 * sizeof(double));
    if (q) memcpy(q, p->q, 4 * sizeof(double));
    if (U) memcpy(U, p->U, 3 * sizeof(double));
    if (W) memcpy(W, p->W, 3 * sizeof(double));
    return 0;
}

int or_get_force_torque(const or_sim* s, int id, double F[3], double T[3]) {
    if (id < 0 || id >= s->np) return -1;
    memcpy(F, s->p[id].F, 3 * sizeof(double));
    memcpy(T, s->p[id].T, 3 * sizeof(double));
    return 0;
}

int or_get_aux(const or_sim* s, int id, double* M, double* dm, double P[3], double L[3], int* nlinks) {
    const opart* p;
    if (id < 0 || id >= s->np) return -1;
    p = &s->p[id];
    if (M) *M = p->M;
    if (dm) *dm = p->dm;
    if (P) memcpy(P, p->Pp, 3 * sizeof(double));
    if (L) memcpy(L, p->Lp, 3 * sizeof(double));
    if (nlinks) *nlinks = p->nlinks;
    return 0;
}

int or_get_zeta(const or_sim* s, int id, double z[36]) {
    if (id < 0 || id >= s->np) return -1;
    memcpy(z, s->p[id].zeta, 36 * sizeof(double));
    return 0;
}

int or_get_links(const or_sim* s, int id, uint32_t* site, uint8_t* dir, int cap) {
    const opart* p;
    int k;
    if (id < 0 || id >= s->np) return -1;
    p = &s->p[id];
    if (cap < p->nlinks) return p->nlinks;
    for (k = 0; k < p->nlinks; k++) {
        site[k] = (uint32_t)p->lsite[k];
        dir[k] = (uint8_t)p->ldir[k];
    }
    return p->nlinks;
}

void or_get_mask(const or_sim* s, uint16_t* owner) {
    int st;
    for (st = 0; st < s->n; st++)
        owner[st] = s->node[st] < 0 ? 0xFFFF : (uint16_t)s->node[st];
}

void or_get_fields(const or_sim* s, double* rho, double* u) {
    int st;
    for (st = 0; st < s->n; st++) {
        double r = 0, v[3] = {0, 0, 0};
        if (s->node[st] == 0) moments(s->q, &s->f[st * s->q], &r, v);
        if (rho) rho[st] = r;
        if (u) {
            u[3 * st] = v[0];
            u[3 * st + 1] = v[1];
            u[3 * st + 2] = v[2];
        }
    }
}

/* Neumaier-compensated running sum, so that conservation checks see the
   method's error and not the error of summing ~10^6 terms */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

double or_get_mass(const or_sim* s) {
    nsum m = {0.0, 0.0};
    int st, i, pid;
    for (st = 0; st < s->n; st++) {
        if (s->node[st] == 0)
            for (i = 0; i < s->q; i++) nadd(&m, s->f[st * s->q + i]);
        else if (s->node[st] > 0)
            nadd(&m, s->rho0); /* particle node counted at the rest density (R9) */
    }
    for (pid = 0; pid < s->np; pid++) nadd(&m, s->p[pid].dm);
    return m.s + m.c;
}

void or_get_momentum(const or_sim* s, double P[3]) {
    nsum a[3] = {{0, 0}, {0, 0}, {0, 0}};
    int st, i;
    for (st = 0; st < s->n; st++)
        if (s->node[st] == 0)
            for (i = 0; i < s->q; i++) {
                double fi = s->f[st * s->q + i];
                nadd(&a[0], fi * CX[i]);
                nadd(&a[1], fi * CY[i]);
                nadd(&a[2], fi * CZ[i]);
            }
    for (i = 0; i < 3; i++) P[i] = a[i].s + a[i].c;
}

long long or_get_step(const or_sim* s) { return s->step; }
int or_overlap_count(const or_sim* s) { return s->overlaps; }

void or_get_f(const or_sim* s, double* out) { memcpy(out, s->f, sizeof(double) * (size_t)s->n * s->q); }
void or_set_f(or_sim* s, const double* in) { memcpy(s->f, in, sizeof(double) * (size_t)s->n * s->q); }

void or_stream_only(or_sim* s) {
    int st;
    memcpy(s->fs, s->f, sizeof(double) * (size_t)s->n * s->q);
    for (st = 0; st < s->n; st++) {
        int x = st % s->nx, y = (st / s->nx) % s->ny, z = st / (s->nx * s->ny), i;
        for (i = 0; i < s->q; i++) {
            int src = site_of(s, wrapi(x - CX[i], s->nx), wrapi(y - CY[i], s->ny),
                              wrapi(z - CZ[i], s->nz));
            s->f[st * s->q + i] = s->fs[src * s->q + i];
        }
    }
}
