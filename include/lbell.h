/*
 * lbell.h - C ABI of the MI355X (gfx950) lattice Boltzmann library for rigid
 * ellipsoidal particles.
 *
 * Method: Thampi, Stratford, Henrich, "Simulating dynamics of ellipsoidal
 * particles using lattice Boltzmann method" (arXiv 2403.05443).  One call of
 * lb_step advances every box by the algorithm of the paper's Appendix A:
 *   collide (Sec. II.A) -> stream, skipping links into solid nodes ->
 *   velocity-independent force/torque F0, T0 (eqs. F0, T0) ->
 *   lab-frame inertia I(t) and dI/dt (eqs. Irot, Irotdiff) ->
 *   implicit 6x6 solve for U(t+1), Omega(t+1) (eqs. Fdiscrete, Tdiscrete) ->
 *   link bounce-back with moving-boundary term (eqs. fb, ub / ubsquirmer) ->
 *   position and quaternion update (eqs. posupdate, qnplus0, qnplus1) ->
 *   remap of solid/fluid/boundary nodes (eq. ellipsoidsurface) ->
 *   drag matrices zeta (eqs. drag1-drag4).
 *
 * Conventions (all of them are fixed by this header):
 *  - Lattice units: dx = dt = 1, rho0 = 1, c_s^2 = 1/3.  D3Q19 velocity order
 *      0:(0,0,0) 1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1)
 *      6:(0,0,-1) 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0) 11:(1,0,1)
 *      12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1) 15:(0,1,1) 16:(0,-1,-1)
 *      17:(0,1,-1) 18:(0,-1,1); the opposite of an odd i is i+1.
 *      Weights 1/3 (rest), 1/18 (axis), 1/36 (diagonal).  D3Q27 continues
 *      19:(1,1,1) 20:(-1,-1,-1) 21:(1,1,-1) 22:(-1,-1,1) 23:(1,-1,1)
 *      24:(-1,1,-1) 25:(-1,1,1) 26:(1,-1,-1), weights 8/27 (rest), 2/27
 *      (axis), 1/54 (edge), 1/216 (corner).  Link codes and the direction
 *      arguments below use these indices.
 *  - Nodes sit at integer coordinates 0..n-1; site index = x + nx*(y + ny*z).
 *  - Quaternions are Hamilton, scalar first, rotating body to lab
 *    (s_lab = q s_body q^-1, Sec. II.D); Omega is in the lab frame.
 *  - Body axes: semi-axis a lies along body x, b along body y, c along body z.
 *  - A node is solid when (x-x_c)^T A (x-x_c) < 1 (strict), evaluated with the
 *    minimum-image separation in every periodic direction.
 *  - Every call returns lb_status; 0 is success, negative values are errors.
 *    Nothing throws or aborts across this boundary.  A context is not
 *    thread-safe; use one per host thread.
 *  - Device memory is owned by the caller: lb_init receives one device
 *    buffer (the arena) and a hipStream_t; the library never allocates
 *    device memory and never frees the arena.  Host pointers passed in are
 *    read (or written) during the call only.
 */
#ifndef LBELL_H
#define LBELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lb_status;
#define LB_OK          0
#define LB_EINVAL     -1   /* bad argument or configuration                     */
#define LB_ENOMEM     -2   /* arena too small, or a fixed capacity exhausted     */
#define LB_EDEVICE    -3   /* a HIP runtime call failed                          */
#define LB_ESTATE     -4   /* call not valid in the current state               */
#define LB_EOVERLAP   -5   /* particle overlaps another particle or a wall      */
#define LB_ENONFINITE -6   /* non-finite value, singular 6x6 system, or |U|>0.5 */
#define LB_ERANGE     -7   /* caller buffer too small (required size returned)  */
#define LB_EIO        -8   /* checkpoint file could not be read or written      */

/* Collision operators (Sec. II.A). */
#define LB_BGK 0   /* single relaxation time: f* = f - (f - f_eq)/tau                  */
#define LB_TRT 1   /* two relaxation times; tau+ = tau, Lambda = (tau+-1/2)(tau--1/2)  */
#define LB_REG 2   /* hydrodynamic (stress) modes relaxed with tau, non-hydrodynamic
                      (ghost) modes relaxed instantaneously (end of Sec. II.A)         */

/* Population storage.  All but LB_FP64 store deviations f_i - w_i*rho0; the
 * half-precision formats store 2^scale_log2 * (f_i - w_i*rho0).  Collision
 * arithmetic is FP64 for LB_FP64 and FP32 otherwise; particle quantities are
 * always FP64. */
#define LB_FP64 0
#define LB_FP32 1
#define LB_FP16 2
#define LB_BF16 3

/* Rotational update (Sec. II.D, eq. Tdiscrete).  The implicit step solves
 * (I + dI) Omega(t+1) - I Omega(t) = T + T_ext for Omega(t+1), I = I(t) the
 * lab-frame inertia; the modes differ in dI:
 *   LB_ROT_ANALYTIC  dI = [Omega(t)]x I - I [Omega(t)]x, the analytic rate
 *   LB_ROT_FD        dI = I(t) - I(t-1), the backward difference over the
 *                    orientations of the last two steps (I(t-1) = I(t) on
 *                    the step after a particle is added)
 *   LB_ROT_PC        predictor-corrector: the analytic solve predicts
 *                    Omega(t+1), whose mean with Omega(t) rotates q(t) to q*;
 *                    the rotational rows are solved again with I + dI
 *                    replaced by I(q*), the same right-hand side.
 * All three agree for a sphere; the paper found no difference between the
 * first two. */
#define LB_ROT_ANALYTIC 0
#define LB_ROT_FD       1
#define LB_ROT_PC       2

typedef struct lb_config {
    int    lattice;         /* 19 (D3Q19, default) or 27 (D3Q27: the eight corner
                               vectors appended as directions 19-26, each followed by
                               its opposite; Sec. III.A, Fig. 3d)                      */
    int    collision;       /* LB_BGK, LB_TRT or LB_REG                                */
    double tau;             /* relaxation time (TRT: tau+), nu = (tau - 1/2)/3, > 1/2  */
    double magic;           /* TRT Lambda; default 3/16                                */
    int    storage;         /* LB_FP64 / LB_FP32 / LB_FP16 / LB_BF16                   */
    int    scale_log2;      /* half formats: storage scale exponent; 0 = derive from
                               velocity_scale as floor(log2(0.25/(velocity_scale/6)))  */
    double velocity_scale;  /* largest fluid speed expected; default 1e-3              */
    double rho0;            /* mean density; must be 1                                 */
    int    counterforce;    /* 1: a uniform force density g = -sum(F_ext)/N (N = non-wall
                               nodes of the box) on all matter: every fluid node, and
                               every particle by its solid-node count, so that total
                               momentum stays zero (default 0)                        */
    int    max_particles;   /* particle capacity over all boxes (default 1 per box);
                               at most 65534 (the node map holds id + 1 in 16 bits)    */
    double max_semi_axis;   /* largest semi-axis any particle may have (default 8)     */
    int    rotation;        /* inertia term of the rotational update (Sec. II.D):
                               LB_ROT_ANALYTIC (default), LB_ROT_FD or LB_ROT_PC        */
    int    monitor_period;  /* steps between the checks of warm-started boxes (see
                               lb_warm_start); 0 = the default, 25                      */
} lb_config;

typedef struct lb_box {
    int    nx, ny, nz;      /* box edge lengths, each >= 4                             */
    int    walls;           /* 0: periodic in y; 1: solid walls at y=0 and y=ny-1,
                               moving with wall_lo / wall_hi (bounce-back links)       */
    double wall_lo[3];      /* velocity of the wall layer y = 0                        */
    double wall_hi[3];      /* velocity of the wall layer y = ny-1                     */
    int    init;            /* 0: fluid at rest; 1: Couette profile between the walls  */
} lb_box;

typedef struct lb_ctx lb_ctx;

/* Fills *cfg with defaults: D3Q19, BGK, tau = 1, magic = 3/16, FP32 storage,
 * rho0 = 1, no counter-force, max_semi_axis = 8, max_particles = 0 (meaning
 * one per box at lb_init). */
lb_status lb_config_default(lb_config* cfg);

/* Device bytes lb_init needs for this configuration and box list, or 0 if the
 * arguments are invalid.  boxes: host array of nboxes entries. */
size_t lb_arena_bytes(const lb_config* cfg, int nboxes, const lb_box* boxes);

/* Creates a context over nboxes independent boxes.  dev_arena: device buffer
 * of at least lb_arena_bytes() bytes, 256-byte aligned, owned by the caller
 * and kept alive until lb_destroy.  hip_stream: the hipStream_t all work is
 * enqueued on (NULL = the default stream).  Populations are initialised to
 * f_eq(rho0, u0) with u0 = 0, or the wall-driven Couette profile (init = 1),
 * including its first-order non-equilibrium part.  Environment variables
 * read here: LBELL_K1_VARIANT picks the initial collide-stream variant (see
 * lb_autotune); LBELL_FUSED=0 runs boxes that hold one particle through the
 * three-kernel particle phase as well; LBELL_BAND=0 makes every remap rescan
 * test the particle's whole window (by default a rescan between full tests
 * tests only the nodes the last full test found within one node of the
 * surface; the results are the same); LBELL_OVERLAP=1 selects the
 * two-stream schedule.  Synchronises the stream. */
lb_status lb_init(const lb_config* cfg, int nboxes, const lb_box* boxes,
                  void* dev_arena, size_t arena_bytes, void* hip_stream,
                  lb_ctx** out);

/* Adds a rigid ellipsoid (Sec. II.B, eq. ellipsoidsurface) to box `box`.
 * centre: lab position (any real value; wrapped into the box).  semi_axes:
 * (a, b, c) > 0 along body x, y, z.  quat: orientation, normalised if
 * | |q| - 1 | <= 1e-6, else LB_EINVAL.  The particle density defaults to rho0,
 * so its mass is M = rho0 * 4/3 pi a b c and its body inertia is
 * diag(M(b^2+c^2)/5, M(a^2+c^2)/5, M(a^2+b^2)/5) (Sec. II.D).  Nodes inside
 * become solid and their fluid is discarded; boundary links and drag
 * matrices are built.  LB_EINVAL if 2*max(a,b,c)+2 exceeds a box dimension
 * or max(a,b,c) > cfg.max_semi_axis; LB_EOVERLAP if a node would belong to
 * another particle or a wall; LB_ENOMEM when the capacity is exhausted.
 * *id receives a dense particle id (0, 1, ...).  Synchronises. */
lb_status lb_add_ellipsoid(lb_ctx* ctx, int box, const double centre[3],
                           const double semi_axes[3], const double quat[4],
                           int* id);

/* Constant external force and torque on particle id (lab frame); they enter
 * the right-hand sides of eqs. Fdiscrete and Tdiscrete. */
lb_status lb_set_external(lb_ctx* ctx, int id, const double F[3], const double T[3]);

/* Spheroidal squirmer slip (Sec. III.D, eqs. squirmer, ubsquirmer): the
 * boundary velocity gains u_s = -B1 (s.e) s - B2 zeta (s.e) s, with e the body
 * x axis.  Requires b == c.  B1 = B2 = 0 switches it off. */
lb_status lb_set_squirmer(lb_ctx* ctx, int id, double B1, double B2);

/* Overwrites the particle's translational and angular velocity (lab frame).
 * LB_EINVAL unless |U| + |W| max(a, b, c) <= 0.5 (the surface-speed limit
 * that every solved velocity obeys: a boundary point moves less than half a
 * node per step, which the remap window relies on). */
lb_status lb_set_velocity(lb_ctx* ctx, int id, const double U[3], const double W[3]);

/* Particle density (default rho0); rescales M and the body inertia. */
lb_status lb_set_particle_density(lb_ctx* ctx, int id, double rho_p);

/* Enqueues n time steps (Appendix A, steps 1-10) of every box on the stream
 * and returns without waiting.  Device-side errors (overlap, non-finite
 * velocity, singular system, capacity overflow) are latched and reported by
 * the next synchronising call. */
lb_status lb_step(lb_ctx* ctx, int n);

/* Runs n steps exactly as lb_step does (plain launches), timing each
 * collide-stream launch with HIP events bound to the kernel's own start and
 * end, and each particle phase with events recorded on the stream around its
 * launches; *ms_collide and *ms_particle receive the summed GPU durations in
 * milliseconds (either may be NULL).  Synchronises. */
lb_status lb_profile_step(lb_ctx* ctx, int n, double* ms_collide, double* ms_particle);

/* Tuner: times every applicable collide-stream variant inside `reps` real
 * time steps each (after one warm-up step per variant) and keeps the fastest
 * for this context.  Variants:
 *   0  generic 256-site tiles, one block per tile
 *   1  row-wave kernel (single box with nx = 64, 128 or 256)
 *   2  row-wave kernel with non-temporal stores (same condition)
 *   3  generic tiles, XCD-chunked block order
 *   4  generic, two tiles per block          5  the same, XCD-chunked
 *   6  generic, XCD-chunked persistent grid (8 blocks per compute unit)
 *   7  the same with two tiles per block
 *   8  generic, four tiles per block, XCD-chunked
 *   9  generic, XCD-chunked, non-temporal stores
 *  10  generic, two tiles per block, XCD-chunked, non-temporal stores
 *  11  in place: one population buffer, alternating an even step (each
 *      node reads and rewrites its own slots) and an odd step (gather from
 *      and scatter to the neighbours); half the population memory
 *  12  in place, XCD-chunked     13  in place, two tiles per block, XCD-chunked
 *  14  in place, XCD-chunked, non-temporal stores
 *  15  generic, XCD-grouped block order (each XCD takes groups of 16
 *      consecutive tiles, the XCDs' groups alternating), non-temporal stores
 * Moving between the two-buffer variants (0-10, 15) and the in-place ones
 * (11-14) permutes the stored populations into the other layout exactly.
 * With the two-stream schedule only 0-2 apply.  All variants give identical
 * bits, so the 2 x (applicable variants) x (reps + 2) steps the tuner takes
 * (two sweeps over the variants; in each, two untimed and reps timed steps
 * per variant, and a variant counts with the smaller of its two means) are
 * ordinary steps of the simulation: the step counter advances by that many.
 * *variant and *ms_best (milliseconds per collide-stream launch, HIP events
 * around each launch) may be NULL.  Synchronises. */
lb_status lb_autotune(lb_ctx* ctx, int reps, int* variant, double* ms_best);

/* Graph replay.  With steps > 0, lb_step runs whole groups of `steps` time
 * steps as one HIP graph launch each (the kernels of the group are captured
 * on first use, on a private stream, and replayed on the context's stream;
 * a capture is redone when the particle count, the collide-stream variant or
 * the buffer parity differs from the captured one) and the remainder as
 * plain launches.  The captured kernels clear what they need themselves (no
 * memset nodes).  steps = 0 (the default) launches every kernel directly.
 * LB_ESTATE with the two-stream schedule; LB_EINVAL for steps < 0. */
lb_status lb_set_graph(lb_ctx* ctx, int steps);

/* Bandwidth reference: copies `bytes` (a multiple of 16, both pointers
 * 16-byte aligned device memory owned by the caller) from src to dst `reps`
 * times on hip_stream with 16-byte accesses (one per thread, a grid covering
 * the buffer), after one warm-up copy, and
 * returns the achieved read+write rate in GB/s (2 * bytes per copy).  Needs
 * no context.  Synchronises the stream. */
lb_status lb_bandwidth_probe(void* dst, const void* src, size_t bytes, void* hip_stream, int reps,
                             double* gbs);

/* Waits for the stream; returns the first latched device error, if any. */
lb_status lb_sync(lb_ctx* ctx);

/* Hydrodynamic force and torque on particle id over the last step
 * (eqs. Fsplit, Tsplit): F = F0 + Fslip - zeta_FU U(t+1) - zeta_FW W(t+1)
 * plus the impulse of nodes covered or uncovered in the previous remap;
 * torque about the centre.  External loads are not included.  Synchronises. */
lb_status lb_get_force_torque(lb_ctx* ctx, int id, double F[3], double T[3]);

/* Position (unwrapped: initial centre plus accumulated displacement),
 * orientation, velocity and angular velocity of particle id.  Any output
 * pointer may be NULL.  Synchronises. */
lb_status lb_get_particle(lb_ctx* ctx, int id, double x[3], double q[4],
                          double U[3], double W[3]);

/* Book-keeping of particle id: mass M, undistributed mass dm of covered and
 * uncovered nodes (returned to the fluid at the next bounce-back), pending
 * momentum P[3] and angular momentum L[3] of those nodes (added to the next
 * implicit solve), and the current number of boundary links.  Any output
 * pointer may be NULL.  Synchronises. */
lb_status lb_get_particle_aux(lb_ctx* ctx, int id, double* M, double* dm,
                              double P[3], double L[3], int* nlinks);

/* Boundary links (x, b) of particle id: x fluid, x + c_b solid (Sec. II.B).
 * site[k] is the site index of x, dir[k] is b (1..18 on D3Q19, 1..26 on
 * D3Q27).  Order: deterministic, not sorted.  If cap < the number of links, nothing is copied, *n is set and
 * LB_ERANGE returned.  Synchronises. */
lb_status lb_get_links(lb_ctx* ctx, int id, uint32_t* site, uint8_t* dir,
                       int cap, int* n);

/* Node map of box: 0 = fluid, id+1 = solid node of particle id, 0xFFFF = wall.
 * owner: host array of nx*ny*nz entries.  Synchronises. */
lb_status lb_get_mask(lb_ctx* ctx, int box, uint16_t* owner);

/* Density and velocity of the (pre-collision) fluid at every site of box,
 * rho[site], u[3*site + k]; solid and wall sites report rho = 0, u = 0.
 * Either pointer may be NULL.  Synchronises. */
lb_status lb_get_fields(lb_ctx* ctx, int box, double* rho, double* u);

/* Conserved mass of box: sum of rho over fluid nodes, rho0 for every node
 * inside a particle (a node changing side carries rho0 with it), plus the
 * pending excess mass dm of its particles.
 * Momentum: sum of rho*u over fluid nodes (particles not included).
 * Synchronises. */
lb_status lb_get_mass(lb_ctx* ctx, int box, double* mass);
lb_status lb_get_momentum(lb_ctx* ctx, int box, double P[3]);

/* Counts non-finite populations on fluid nodes of box.  Synchronises. */
lb_status lb_check_finite(lb_ctx* ctx, int box, long long* count);

/* Number of completed steps. */
lb_status lb_get_step(lb_ctx* ctx, long long* step);

/* Checkpoint: every population, node map, link list and particle record plus
 * the step counter, to a binary file; lb_load restores it into a context made
 * with the same configuration and boxes (in either population layout: the
 * file records its own, and the load converts to the one the context's
 * collide-stream variant uses).  LB_EIO on file errors, LB_EINVAL on
 * a mismatching file (another configuration, or a file format version other
 * than this library's, currently 3).  Synchronise. */
lb_status lb_save(lb_ctx* ctx, const char* path);
lb_status lb_load(lb_ctx* ctx, const char* path);

/* Test hook: sets the pre-collision population dir of site in box to
 * w_dir*rho0 + value (so value is the deviation; NaN allowed).  Synchronises. */
lb_status lb_debug_poke(lb_ctx* ctx, int box, int site, int dir, double value);

/* Releases host resources of ctx (not the arena).  Synchronises. */
lb_status lb_destroy(lb_ctx* ctx);

/* ------------------------------------------------------------------------
 * Learned warm start.  The paper has no learned part: the surrogate and the
 * warm start serve to reach the steady state of a run in fewer steps.  A
 * small network maps a particle's shape, confinement and load to its steady
 * velocities; a run then starts from those velocities and from the creeping
 * flow around the particle instead of from rest.
 *
 * Network: 8 -> 64 -> 64 -> 6, tanh hidden layers, linear output; 5126 FP32
 * parameters, flat in the order W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[6][64], b3[6].  Products run on the matrix cores with bfloat16 operands
 * (inputs, weights, hidden activations, back-propagated errors) and FP32
 * accumulation.  Loss: mean squared error over the n x 6 outputs.  Training:
 * Adam (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master
 * parameters.
 *
 * Inputs and outputs (all FP32, row-major, host memory owned by the caller):
 * for a particle with semi-axes (a, b, c), orientation R(q), external load
 * (F, T), equal-volume radius Req = (abc)^(1/3), load scale
 * s = sqrt(|R^T F|^2 + |R^T T|^2 / Req^2) and L^3 its box's volume per
 * particle (the box's volume over its number of particles),
 *   x = (ln(a / sqrt(bc)), a / L, R^T F / s, R^T T / (Req s)),
 *   y = (U_body 6 pi mu Req / s, Omega_body 8 pi mu Req^2 / s),  mu = rho0 nu.
 * A squirmer (lb_set_squirmer, B1 != 0) carries no load of its own: its body
 * frame load gains the equivalent propulsive force F_eff along its axis,
 * the drag of a prolate spheroid translating along its axis at the free
 * swimming speed (Sec. III.D, eq. squirmervel),
 *   F_eff = 6 pi mu a X^A(e) U_s,  U_s = B1 e^-1 (e^-1 - (e^-2 - 1) arcoth(1/e)),
 *   X^A(e) = (8/3) e^3 / (-2 e + (1 + e^2) ln((1 + e) / (1 - e))),
 * e = sqrt(1 - b c / a^2) (1 and 2 B1 / 3 for a sphere); the start field of
 * the warm start stays that of the external loads alone.
 * ------------------------------------------------------------------------ */
typedef struct lbs lbs;

/* Device bytes a surrogate needs to hold up to max_samples samples. */
size_t lbs_arena_bytes(int max_samples);

/* Creates a surrogate in a caller-owned device arena (256-byte aligned, kept
 * alive until lbs_destroy) working on hip_stream.  Parameters start at zero:
 * set them with lbs_set_params.  LB_ENOMEM if bytes is too small. */
lb_status lbs_create(int max_samples, void* dev_arena, size_t bytes, void* hip_stream, lbs** out);

/* Copies 5126 parameters in (and resets the Adam moments and step count) or
 * out.  Synchronise. */
lb_status lbs_set_params(lbs* s, const float* params);
lb_status lbs_get_params(lbs* s, float* params);

/* `epochs` passes over the n samples (X: n x 8, Y: n x 6) in their given
 * order, in mini-batches of `batch` (the last one may be shorter), one Adam
 * step of size lr per mini-batch.  *loss (may be NULL) receives the mean
 * squared error of the last epoch accumulated over its mini-batches.
 * LB_EINVAL for n < 1, n > max_samples, batch < 1 or epochs < 1.
 * Synchronises. */
lb_status lbs_train(lbs* s, const float* X, const float* Y, int n, int epochs, int batch, float lr,
                    float* loss);

/* Network outputs for n inputs (X: n x 8 -> Y: n x 6).  Synchronises. */
lb_status lbs_predict(lbs* s, const float* X, int n, float* Y);

/* Loss and its gradient with respect to the 5126 parameters over n samples
 * (for gradient checks); grads and loss may be NULL.  Synchronises. */
lb_status lbs_grad(lbs* s, const float* X, const float* Y, int n, float* grads, float* loss);

/* Releases host resources of s (not the arena). */
lb_status lbs_destroy(lbs* s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the loss
 * and gradient of lbs_grad, computed by the same kernels in the same order,
 * with no surrogate object, no arena and no allocation of any kind.  All
 * pointers are device memory owned by the caller: params (5126 floats, the
 * order above), X (n x 8), Y (n x 6), grads (5126 floats, written), loss (one
 * float, written; may be NULL).  Work is enqueued on hip_stream (a stream of
 * the current device) and the call returns without waiting.  The per-tile
 * partial gradients live in a fixed device array of the library (5.3 MB,
 * one per device, kept until the process ends): n above
 * LBS_NOALLOC_MAX_SAMPLES is rejected with LB_EINVAL, as are NULL pointers
 * and n < 1.  Every call on a device shares that array, so calls that overlap
 * on one device (other streams, other host threads) race; order them on one
 * stream. */
#define LBS_NOALLOC_MAX_SAMPLES 4096
lb_status lbs_grad_noalloc(const float* params, const float* X, const float* Y, int n, float* grads, float* loss,
                           void* hip_stream);

/* Warm start of the particles of box `box` (every box for box = -1): the
 * surrogate predicts each particle's steady velocities from its current state
 * and external load; they are set as the particles' velocities (a prediction
 * above the surface-speed limit of lb_set_velocity is scaled down to it), and
 * the fluid of the box is then started as lb_stokes_start does.  pred (may be
 * NULL) receives the predicted lab-frame (U, Omega) of every particle, 6
 * doubles per particle id (only those of the box are meaningful).
 *
 * With tol > 0 the box is then watched on the device, every
 * cfg.monitor_period steps of lb_step.  W0 = max over the box's particles of
 * ceil(2 a^2 / nu) (a the largest semi-axis) is the time in which a particle
 * sheds the error of its start.  The first check at least W0 / 4 steps after
 * the warm start records the box's flow energy (the sum of |j|^2 over its
 * fluid nodes, j the momentum density) and its particles' velocities
 * V = (U, a Omega); the first check at least W0 steps after it compares with
 * them (the residuals: the relative changes since then) and with the
 * prediction, and decides the box.  The box misses when more than a quarter
 * of its particles are further than tol from their predictions (a box of
 * one to three particles: when any is):
 *   LB_WARM_ACCEPTED     no miss;
 *   LB_WARM_FALLBACK     a miss while a residual still exceeds tol: the
 *                        surrogate's start has failed, and the box falls back
 *                        to the plain method: its fluid and particles are
 *                        reset to rest and the run goes on from there (the
 *                        steps so far are spent);
 *   LB_WARM_STEADY_MISS  a miss with both residuals below tol: the run is
 *                        steady away from the prediction; it is kept, and its
 *                        samples (lb_surrogate_sample) belong in the training
 *                        data.
 * tol <= 0 leaves the box unwatched.  Needs np <= the surrogate's
 * max_samples; LB_EINVAL for boxes with walls or box out of range.
 * Synchronises. */
#define LB_WARM_OFF         0
#define LB_WARM_PENDING     1
#define LB_WARM_ACCEPTED    2
#define LB_WARM_FALLBACK    3
#define LB_WARM_STEADY_MISS 4
lb_status lb_warm_start(lb_ctx* ctx, int box, lbs* s, double tol, double* pred);

/* State of the warm-start monitor of every box (host arrays of nboxes
 * entries, either may be NULL): status (LB_WARM_*) and the step at which it
 * was decided (-1 while pending or unwatched).  Synchronises. */
lb_status lb_warm_status(lb_ctx* ctx, int* status, long long* decided_step);

/* Starts the fluid of every box from the creeping flow its particles'
 * external loads drive.  Each node gets the sum over the box's particles of
 * the free-space flow the load (F_ext, T_ext) drives, at minimum-image
 * offsets, rigid motion inside the body: for a prolate spheroid (a > b = c)
 * the exact solution (Chwang & Wu's singularities on the focal segment, the
 * body moving with the velocities of eq. drag4's resistance functions); for
 * any other shape the sphere of the equal-volume radius R moving with
 * F_ext / (6 pi mu R) and turning with T_ext / (8 pi mu R^3) (Stokes'
 * solution and the rotlet).  Its Fourier modes |n_i| <= 2 of the box (fewer
 * along an edge shorter than 5) are replaced by those of the periodic flow
 * of the same loads (the force spread as the traction on the translating
 * ellipsoid, the torque as that on the rotating prolate spheroid, or over
 * the sphere of radius R for any other body), so
 * the box's slowest shear modes start at their steady values; the same for
 * the flow's pressure p (the Stokeslets' and stresslets'; the periodic
 * modes -i (k.f) / k^2 of the force density f).  A fluid node gets the
 * density rho0 + 3 (p - pbar), pbar the mean over the box's fluid nodes, and
 * the fluid nodes then lose the uniform velocity that makes the box's total
 * momentum (fluid sum rho u plus the particles' M U) zero; nodes inside a
 * particle have rho0 and move rigidly with its current U, Omega.  Every node
 * is set to the second-order equilibrium at its density and velocity (mass
 * is unchanged).  The free flow is staged in the population buffer that
 * does not hold the state (no allocation).  LB_EINVAL if a box has walls.
 * Synchronises. */
lb_status lb_stokes_start(lb_ctx* ctx);

/* Training sample of every particle at its current state: the surrogate's
 * inputs (X, 8 floats per particle id) and its normalised body-frame
 * response at the particle's current velocities (Y, 6 floats per particle:
 * the inverse of the output scaling above; zero for an unloaded particle).
 * Synchronises. */
lb_status lb_surrogate_sample(lb_ctx* ctx, float* X, float* Y);

/* Bulk read-back of particles [first, first + count): x (unwrapped), q, U, W
 * as 3, 4, 3, 3 doubles per particle (any pointer may be NULL).
 * Synchronises. */
lb_status lb_get_particles(lb_ctx* ctx, int first, int count, double* x, double* q, double* U, double* W);

/* Static text for a status code. */
const char* lb_status_str(lb_status s);

/* Text of the last error recorded in ctx ("" if none). */
const char* lb_last_error(lb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBELL_H */
