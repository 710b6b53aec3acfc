/*
 * lbe_oracle.h - FP64 CPU oracle for the lattice Boltzmann method with rigid
 * ellipsoidal particles of Thampi, Stratford & Henrich (arXiv 2403.05443).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; it is
 * called from the test-suite, from the package smoke check and from the CPU
 * baseline leg of the benchmark, never from the product path.  It shares no
 * source, header, table or helper with the HIP library.
 *
 * Storage: full populations f_i (not deviations), one AoS array of q doubles
 * per node (q = 19 for D3Q19, 27 for D3Q27), explicit separate collision and streaming loops, the node map as
 * an int per site (0 fluid, p+1 solid node of particle p, -1 wall).
 */
#ifndef LBE_ORACLE_H
#define LBE_ORACLE_H
#include <stdint.h>

typedef struct or_sim or_sim;

/* collision: 0 BGK, 1 TRT (magic = Lambda), 2 ghost modes relaxed at once */
or_sim* or_create(int nx, int ny, int nz, int collision, double tau, double magic,
                  int walls, const double ulo[3], const double uhi[3], int init,
                  int counterforce);
/* the same on the D3Q19 (lattice = 19) or D3Q27 (27) velocity set; NULL
   for any other lattice */
or_sim* or_create_q(int nx, int ny, int nz, int collision, double tau, double magic,
                    int walls, const double ulo[3], const double uhi[3], int init,
                    int counterforce, int lattice);
/* treatment of the inertia in the rotational equation (Sec. II.D): 0 the
   analytic dI/dt of eq. Irotdiff with I(t) (default); 1 dI/dt as the finite
   difference (I(t) - I(t - dt)) / dt; 2 predictor-corrector for I(t + dt):
   the solve with mode 0 predicts Omega(t + dt), the orientation it gives
   yields I(t + dt), and the rotational rows are solved again as
   I(t + dt) Omega(t + dt) - I(t) Omega(t) = dt T.  -1 for another mode. */
int     or_set_rotation(or_sim* s, int mode);
void    or_destroy(or_sim* s);
int     or_add_ellipsoid(or_sim* s, const double centre[3], const double axes[3],
                         const double quat[4]);
int     or_set_external(or_sim* s, int id, const double F[3], const double T[3]);
int     or_set_squirmer(or_sim* s, int id, double B1, double B2);
int     or_set_velocity(or_sim* s, int id, const double U[3], const double W[3]);
int     or_set_density(or_sim* s, int id, double rho_p);
int     or_step(or_sim* s, int n);

int     or_get_particle(const or_sim* s, int id, double x[3], double q[4],
                        double U[3], double W[3]);
int     or_get_force_torque(const or_sim* s, int id, double F[3], double T[3]);
int     or_get_aux(const or_sim* s, int id, double* M, double* dm, double P[3],
                   double L[3], int* nlinks);
int     or_get_zeta(const or_sim* s, int id, double z[36]);
int     or_get_links(const or_sim* s, int id, uint32_t* site, uint8_t* dir, int cap);
void    or_get_mask(const or_sim* s, uint16_t* owner);
void    or_get_fields(const or_sim* s, double* rho, double* u);
/* box mass counting every particle node at rho0, plus pending excess (R9) */
double  or_get_mass(const or_sim* s);
void    or_get_momentum(const or_sim* s, double P[3]);
long long or_get_step(const or_sim* s);
int     or_overlap_count(const or_sim* s);

/* raw access for pins: pre-collision populations f[site*q + i] */
void    or_get_f(const or_sim* s, double* out);
void    or_set_f(or_sim* s, const double* in);
/* pins on single pieces of the method */
void    or_equilibrium(double rho, const double u[3], double feq[19]);
void    or_equilibrium_q(int lattice, double rho, const double u[3], double* feq);
void    or_collide_node(const or_sim* s, const double* f, double* out);
void    or_stream_only(or_sim* s);   /* post-collision := f, then stream, no links */
int     or_inside(int nx, int ny, int nz, const double xc[3], const double axes[3],
                  const double q[4], int x, int y, int z);
void    or_inertia_lab(const double q[4], const double Ib[3], double out[9]);
void    or_inertia_dot(const double q[4], const double Ib[3], const double W[3],
                       double out[9]);
int     or_solve6(const double A[36], const double b[6], double x[6]);
void    or_quat_update(const double q[4], const double Wmean[3], double out[4]);
void    or_squirmer_slip(const double axes[3], const double q[4], double B1, double B2,
                         const double d[3], double us[3]);
void    or_lattice(int c[57], double w[19]);
void    or_lattice_q(int lattice, int* c, double* w);
#endif
