"""Runs built on the library: lattices from workload descriptions, training
data for the warm-start surrogate from batched ensembles, its training, and
the comparison of the steps a run needs to reach its steady state from a
plain start (fluid at rest), from the surrogate's warm start, and from a
warm start with the unbounded-fluid closed forms (the control, the same
start without the network).

Every step of the method runs in the HIP library; this module only drives
it (launch sizes, step counts, book-keeping of the sampled velocities) and
shapes the training data.
"""
import math
import time

import numpy as np

from . import lbell, workloads


def build_lattice(W, device="cuda:0"):
    """A Lattice holding workload W (boxes, particles, loads, squirmers)."""
    boxes = [lbell.make_box(*b.shape, walls=b.walls, wall_lo=b.wall_lo, wall_hi=b.wall_hi, init=b.init)
             for b in W.boxes]
    lat = lbell.Lattice(boxes, collision=W.collision, tau=W.tau, magic=W.magic, storage=W.storage,
                        counterforce=W.counterforce, velocity_scale=W.velocity_scale,
                        max_particles=max(1, len(W.particles)), max_semi_axis=W.max_semi_axis,
                        lattice=W.lattice, device=device)
    for p in W.particles:
        pid = lat.add_ellipsoid(p.centre, p.axes, p.quat, box=p.box)
        lat.set_external(pid, p.force, p.torque)
        if p.squirmer != (0.0, 0.0):
            lat.set_squirmer(pid, *p.squirmer)
    return lat


def viscosity(W):
    return (W.tau - 0.5) / 3.0


def slow_time(L, nu):
    """e-folding time of the slowest shear mode of a periodic box of edge L."""
    return L * L / (4 * math.pi ** 2 * nu)


def box_edge(W, i):
    nx, ny, nz = W.boxes[W.particles[i].box].shape
    return (nx * ny * nz) ** (1.0 / 3.0)


# ------------------------------------------------------------ training data --

def ensemble_samples(W, efolds=8.0, graph=50):
    """Runs the ensemble W for `efolds` slow times of its largest box and
    returns the surrogate's inputs and normalised responses of every particle
    at the end, (X (n, 8), Y (n, 6))."""
    lat = build_lattice(W)
    nu = viscosity(W)
    steps = int(math.ceil(efolds * max(slow_time(box_edge(W, i), nu) for i in range(len(W.particles)))))
    lat.set_graph(graph)
    lat.step(steps)
    X, Y = lat.surrogate_sample()
    del lat
    return X.astype(np.float64), Y.astype(np.float64), steps


def augment(X, Y, nrot=8, flip=True, negate=True):
    """Copies of the samples under the symmetries of a spheroid with b = c:
    rotations about its axis (body x) by 2 pi k / nrot and, with flip, the
    half-turn about body z that swaps its ends.  Loads and responses rotate
    together (forces, torques and both velocities transform alike under
    proper rotations); the shape inputs are unchanged.  With negate, each
    copy also with loads and responses reversed: Stokes flow is linear in
    the load, and the normalised inputs and outputs are odd in it."""
    out_x, out_y = [], []
    mats = []
    for k in range(nrot):
        c, s = math.cos(2 * math.pi * k / nrot), math.sin(2 * math.pi * k / nrot)
        Q = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
        mats.append(Q)
        if flip:
            mats.append(np.diag([-1.0, -1.0, 1.0]) @ Q)
    for Q in mats:
        for sg in ((1.0, -1.0) if negate else (1.0,)):
            x, y = X.copy(), Y.copy()
            x[:, 2:5], x[:, 5:8] = sg * (X[:, 2:5] @ Q.T), sg * (X[:, 5:8] @ Q.T)
            y[:, 0:3], y[:, 3:6] = sg * (Y[:, 0:3] @ Q.T), sg * (Y[:, 3:6] @ Q.T)
            out_x.append(x)
            out_y.append(y)
    return np.concatenate(out_x), np.concatenate(out_y)


def shuffle(X, Y, seed):
    """Fisher-Yates permutation drawn from the project generator."""
    g = workloads.SplitMix64(seed)
    idx = np.arange(len(X))
    for i in range(len(idx) - 1, 0, -1):
        j = int(g.next_u64() % (i + 1))
        idx[i], idx[j] = idx[j], idx[i]
    return X[idx], Y[idx]


def train_surrogate(X, Y, seed=2403054430, epochs=1000, batch=256, lr=3e-3, lr_end=3e-5, stages=10, val_frac=0.2):
    """Xavier initialisation, seeded shuffle, 80/20 split, Adam on the GPU with
    the step size lowered geometrically from lr to lr_end over `stages`
    equal parts of the epochs (the moments carry over).  Returns
    (surrogate, info)."""
    X, Y = shuffle(X, Y, seed)
    nval = int(round(val_frac * len(X)))
    Xv, Yv, Xt, Yt = X[:nval], Y[:nval], X[nval:], Y[nval:]
    sur = lbell.Surrogate(max_samples=max(len(X), 64), params=workloads.xavier_params(workloads.SplitMix64(seed)))
    L0 = sur.grad(Xt, Yt)[0]
    per = max(1, epochs // stages)
    for k in range(stages):
        step = lr * (lr_end / lr) ** (k / max(stages - 1, 1))
        Lt = sur.train(Xt, Yt, epochs=per, batch=batch, lr=step)
    Lv = sur.grad(Xv, Yv)[0] if nval else float("nan")
    var = float(np.mean((Yv - Yv.mean(0)) ** 2)) if nval else float("nan")
    return sur, {"samples": len(X), "train": len(Xt), "val": nval, "loss_init": L0, "loss_train": Lt,
                 "loss_val": Lv, "val_target_variance": var}


# ---------------------------------------------------- closed-form control --

def resistance(r):
    """X^A, Y^A, X^C, Y^C of a prolate spheroid of aspect ratio r (Kim &
    Karrila, Microhydrodynamics, Table 3.4); 1 for a sphere."""
    if r < 1 + 1e-6:
        return 1.0, 1.0, 1.0, 1.0
    e = math.sqrt(1 - 1 / (r * r))
    lg = math.log((1 + e) / (1 - e))
    return (8 / 3 * e ** 3 / (-2 * e + (1 + e * e) * lg), 16 / 3 * e ** 3 / (2 * e + (3 * e * e - 1) * lg),
            4 / 3 * e ** 3 * (1 - e * e) / (2 * e - (1 - e * e) * lg),
            4 / 3 * e ** 3 * (2 - e * e) / (-2 * e + (1 + e * e) * lg))


def ellipsoid_resistance(axes, mu, n=200):
    """Translational and rotational resistance of an ellipsoid with
    semi-axes (a1, a2, a3) about its body axes in an unbounded fluid
    (Oberbeck's integrals, as in Jeffery 1922): with
    D(l) = sqrt((a1^2 + l)(a2^2 + l)(a3^2 + l)), chi = int_0^inf dl / D and
    alpha_i = int_0^inf dl / ((a_i^2 + l) D), translation along axis i costs
    16 pi mu / (chi + a_i^2 alpha_i) and rotation about it
    16 pi mu (a_j^2 + a_k^2) / (3 (a_j^2 alpha_j + a_k^2 alpha_k)).  The
    integrals are taken by Gauss-Legendre quadrature after
    l = s^2 (1 - u^2) / u^2 (s = the largest semi-axis), which maps [0, inf)
    to (0, 1] with smooth integrands (dl / D tends to 2 du / s at u = 0)."""
    a2 = np.asarray(axes, float) ** 2
    sc = a2.max()
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wt = 0.5 * w
    lam = sc * (1.0 - u * u) / (u * u)
    jac = 2.0 * sc / u ** 3
    D = np.sqrt((a2[0] + lam) * (a2[1] + lam) * (a2[2] + lam))
    chi = np.sum(wt * jac / D)
    alpha = np.array([np.sum(wt * jac / ((a2[i] + lam) * D)) for i in range(3)])
    trans = 16 * math.pi * mu / (chi + a2 * alpha)
    rot = np.array([16 * math.pi * mu * (a2[j] + a2[k]) / (3 * (a2[j] * alpha[j] + a2[k] * alpha[k]))
                    for j, k in ((1, 2), (0, 2), (0, 1))])
    return trans, rot


def _rot(q):
    q0, q1, q2, q3 = q
    return np.array([[1 - 2 * (q2 * q2 + q3 * q3), 2 * (q1 * q2 - q0 * q3), 2 * (q1 * q3 + q0 * q2)],
                     [2 * (q1 * q2 + q0 * q3), 1 - 2 * (q1 * q1 + q3 * q3), 2 * (q2 * q3 - q0 * q1)],
                     [2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1), 1 - 2 * (q1 * q1 + q2 * q2)]])


def unbounded_velocities(p, nu):
    """Velocities of particle p under its load in an unbounded fluid at rest
    (no periodic images): the Kim-Karrila closed forms for a prolate
    spheroid (a, b, b), a >= b, Oberbeck's integrals for any other
    ellipsoid (rho0 = 1, so mu = nu)."""
    a, b, c = p.axes
    R = _rot(p.quat)
    Fb, Tb = R.T @ np.asarray(p.force, float), R.T @ np.asarray(p.torque, float)
    if b == c and a >= b:
        XA, YA, XC, YC = resistance(a / b)
        Ub = np.array([Fb[0] / XA, Fb[1] / YA, Fb[2] / YA]) / (6 * math.pi * nu * a)
        Wb = np.array([Tb[0] / XC, Tb[1] / YC, Tb[2] / YC]) / (8 * math.pi * nu * a ** 3)
    else:
        trans, rot = ellipsoid_resistance(p.axes, nu)
        Ub, Wb = Fb / trans, Tb / rot
    return R @ Ub, R @ Wb


# --------------------------------------------- domain size and resolution --

def settling_run(W, transient, graph=50, tune=True, sample=50, travel=1.0):
    """Settling velocity of the single particle of workload W, started from
    the closed-form control (unbounded velocities and the periodic Stokes
    start field).  After `transient` steps, U is sampled every `sample` steps
    over two windows in each of which the particle travels about `travel`
    lattice spacings: as the particle moves, nodes change side and the
    velocity jumps by a fraction of a percent (the discrete-shape error of
    the method), so only a mean over such a window is a settled value.
    Returns the mean over the last window, its relative change from the
    window before (drift), the relative spread of the samples in it, and
    the site updates per second of the last window (graph replay, sampling
    included)."""
    import time
    import torch
    nu = viscosity(W)
    p = W.particles[0]
    lat = build_lattice(W)
    if tune:
        lat.autotune(2)  # ordinary steps; the start below replaces fluid and particle velocities
    U0, W0 = unbounded_velocities(p, nu)
    force = np.asarray(p.force, float)
    e = force / np.linalg.norm(force)
    Uc = float(np.asarray(U0, float) @ e)
    every = int(math.ceil(travel / abs(Uc) / sample)) * sample
    lat.set_velocity(0, U0, W0)
    lat.stokes_start()
    lat.set_graph(graph if sample % graph == 0 else sample)
    lat.step(transient)

    def window():
        us = []
        for _ in range(every // sample):
            lat.step(sample)
            us.append(lat.particles()["U"][0].copy())
        return np.array(us)
    Ua = window().mean(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wb = window()
    dt = time.perf_counter() - t0
    del lat
    Ub = wb.mean(0)
    U = float(Ub @ e)
    return {"L": W.boxes[0].shape[0], "U": U, "U_closed": Uc, "error": U / Uc - 1,
            "drift": float(np.linalg.norm(Ub - Ua) / np.linalg.norm(Ub)),
            "spread": float((wb @ e).std() / abs(U)), "steps": transient + 2 * every,
            "mlups": W.sites * every / dt / 1e6, "U_vec": Ub.tolist()}


def drift_superposition(bs=(2.0, 3.0, 4.0), r=3.0, l_over_b=64, alpha_deg=45.0, nu=0.1, U_target=1e-4,
                        storage="fp32", travel=1.0):
    """Lateral drift of an inclined settling spheroid (Sec. III.B, eq. drift)
    against resolution: for semi-axes (r b, b, b) in a periodic box of edge
    l_over_b * b, the drift angle delta of a particle whose axis makes
    alpha with the force (measured: angle between velocity and force), and
    the drift the paper predicts from the settling speeds of the end-on and
    broadside orientations in the same box (linear superposition:
    tan(alpha - delta) = (U_perp / U_par) tan alpha).  The force is scaled
    with b so that the speed (and Reynolds number U a / nu) stays near
    U_target.  Returns one row per b with both angles, their gap and the
    closed form of eq. drift."""
    out = []
    for b in bs:
        L = int(round(l_over_b * b))
        a = r * b
        XA, YA, _, _ = resistance(r)
        force = U_target * 6 * math.pi * nu * a * XA
        runs = {}
        for name, ang in (("inclined", alpha_deg), ("end-on", 0.0), ("broadside", 90.0)):
            W = workloads.settling(L, a, b, "end-on", nu, force, storage)
            # body x at angle ang from the force (lab x), rotating about lab z
            W.particles[0].quat = workloads.quat_axis_angle((0.0, 0.0, 1.0), math.radians(ang))
            runs[name] = settling_run(W, int(4 * a * a / nu), travel=travel)
        F = np.array([1.0, 0.0, 0.0])
        Ui = np.array(runs["inclined"]["U_vec"])
        delta = math.degrees(math.acos(Ui @ F / np.linalg.norm(Ui)))
        Upar, Uperp = runs["end-on"]["U"], runs["broadside"]["U"]
        sup = alpha_deg - math.degrees(math.atan(Uperp / Upar * math.tan(math.radians(alpha_deg))))
        closed = alpha_deg - math.degrees(math.atan(XA / YA * math.tan(math.radians(alpha_deg))))
        out.append({"b": b, "a": a, "L": L, "force": force, "delta_measured": delta, "delta_superposition": sup,
                    "gap": sup / delta - 1, "delta_closed": closed, "U_par": Upar, "U_perp": Uperp,
                    "spread": max(v["spread"] for v in runs.values()),
                    "steps": max(v["steps"] for v in runs.values())})
    return out


def domain_sweep(lengths, a=7.5, b=2.5, nu=0.1, force=2e-3, storage="fp32", transient=None, lattice=19,
                 orientations=("end-on", "broadside"), c=None):
    """Settling velocity against box edge L for both orientations (Fig. 4),
    and for each orientation the fit U(L) = U_inf (1 - k / L) over the boxes
    of edge >= 8a (the leading periodic-image correction), U_inf against the
    closed form of eq. settlingvel."""
    amax = max(a, b, c or 0.0)
    transient = transient or int(4 * amax * amax / nu)
    out = {}
    for orient in orientations:
        rows = [settling_run(workloads.settling(L, a, b, orient, nu, force, storage, lattice, c), transient)
                for L in lengths]
        big = [r for r in rows if r["L"] >= 8 * amax] or rows
        x = np.array([1.0 / r["L"] for r in big])
        y = np.array([r["U"] for r in big])
        A = np.vstack([np.ones_like(x), x]).T
        c0, c1 = np.linalg.lstsq(A, y, rcond=None)[0]
        out[orient] = {"runs": rows, "U_inf_fit": float(c0), "k_fit": float(-c1 / c0),
                       "U_closed": rows[0]["U_closed"], "fit_error": float(c0 / rows[0]["U_closed"] - 1)}
    return out


def resolution_sweep(bs, r=3.0, l_over_b=(32, 64), nu=0.1, force=2e-3, storage="fp32",
                     orientations=("end-on", "broadside"), travel=2.0):
    """Settling velocity against resolution (Fig. 9): semi-axes (r b, b, b)
    for b in bs at the same force (so the same Reynolds number
    F / (6 pi mu nu)), each in two boxes of edge l_over_b * b; the 1/L law
    through the two removes the periodic images, and the extrapolated
    velocity, normalized by that of a sphere of radius b (F / (6 pi mu b)),
    is compared with the closed form of eq. settlingvel."""
    out = {}
    for orient in orientations:
        rows = []
        for bb in bs:
            runs = [settling_run(workloads.settling(int(round(m * bb)), r * bb, bb, orient, nu, force, storage),
                                 int(4 * (r * bb) ** 2 / nu), travel=travel) for m in l_over_b]
            (L1, U1), (L2, U2) = [(q["L"], q["U"]) for q in runs]
            U_inf = (U2 * L2 - U1 * L1) / (L2 - L1)  # U = U_inf (1 - k / L) through both
            norm = force / (6 * math.pi * nu * bb)
            rows.append({"b": bb, "L": [L1, L2], "U": [U1, U2], "U_inf": U_inf, "U_norm": U_inf / norm,
                         "U_closed_norm": runs[0]["U_closed"] / norm, "error": U_inf / runs[0]["U_closed"] - 1,
                         "drift": max(q["drift"] for q in runs), "spread": max(q["spread"] for q in runs)})
        out[orient] = rows
    return out


def jeffery_half_period(L, a=6.0, b=2.0, rate=2e-4, nu=0.1, storage="fp32", chunk=250):
    """Steps the long axis of a spheroid in the flow-gradient plane of an L^3
    wall-bounded shear cell takes to turn by pi (half a Jeffery orbit,
    eq. jeffery; closed form pi (r + 1/r) / rate for r = a / b), with
    linear interpolation of the crossing."""
    W = workloads.jeffery_box(L, a, b, rate, nu, storage)
    lat = build_lattice(W)
    lat.autotune(2)
    lat.set_graph(50 if chunk % 50 == 0 else chunk)
    r = a / b
    T_half = math.pi * (r + 1 / r) / rate
    phi, last, t = 0.0, 0.0, 0
    while True:
        lat.step(chunk)
        t += chunk
        q = lat.particles()["q"][0]
        ex, ey = 1 - 2 * (q[2] ** 2 + q[3] ** 2), 2 * (q[1] * q[2] + q[0] * q[3])  # body x axis in the lab
        ang = math.atan2(ey, ex)
        d = (ang - last + math.pi) % (2 * math.pi) - math.pi
        prev, phi, last = phi, phi + d, ang
        if abs(phi) >= math.pi:
            t_cross = t - chunk + (math.pi - abs(prev)) / (abs(phi) - abs(prev)) * chunk
            break
        if t > 3 * T_half:
            t_cross = float("nan")
            break
    del lat
    return {"L": L, "half_period": t_cross, "closed_form": T_half, "ratio": t_cross / T_half}


def sphere_array_run(L, R=4.0, force=2e-3, steps=None):
    """A sphere of radius R in a periodic L^3 box (BGK, tau = 1, nu = 1/6)
    under a force: a simple-cubic array of spheres, whose velocity
    Hasimoto's expansion gives exactly for small R / L."""
    nu = 1.0 / 6.0
    W = workloads.settling(L, R, R, "end-on", nu, force, "fp64")
    W.collision = "bgk"
    W.tau = 1.0
    return settling_run(W, steps or int(16 * R * R / nu))


# ------------------------------------------------------- steps to steady --

def trajectory(W, start="plain", surrogate=None, steps=1000, every=25, graph=25, tol=0.0, velocities=None):
    """Velocities U of every particle every `every` steps from one of four
    starts: 'plain' (rest), 'surrogate' (lb_warm_start; with tol > 0 its
    boxes are watched on the device and fall back to the plain start when the
    prediction fails), 'control' (closed forms + Stokes start field), 'given'
    (the particles' velocities `velocities` (np, 3), no rotation, + Stokes
    start field: with the steady velocities it tests the field alone).  Returns
    (times, U (nt, np, 3), pred, info) with info holding the start's wall
    time (start_ms) and, for the surrogate start, the device's decision per
    box and the samples (X, Y) of every particle at the end of the run."""
    lat = build_lattice(W)
    pred = None
    info = {}
    lat.sync()
    t0 = time.perf_counter()
    if start == "surrogate":
        pred = lat.warm_start(surrogate, tol=tol)
    elif start == "control":
        nu = viscosity(W)
        pred = np.zeros((len(W.particles), 6))
        for i, p in enumerate(W.particles):
            U, Wv = unbounded_velocities(p, nu)
            lat.set_velocity(i, U, Wv)
            pred[i] = np.concatenate([U, Wv])
        lat.stokes_start()
    elif start == "given":
        for i in range(len(W.particles)):
            lat.set_velocity(i, velocities[i], (0.0, 0.0, 0.0))
        lat.stokes_start()
    lat.sync()
    info["start_ms"] = 1e3 * (time.perf_counter() - t0)
    lat.set_graph(graph)
    times, Us = [], []
    t = 0
    while t < steps:
        lat.step(every)
        t += every
        times.append(t)
        Us.append(lat.particles()["U"].copy())
    if start == "surrogate":
        info["status"], info["decided"] = lat.warm_status()
        info["samples"] = lat.surrogate_sample()
    del lat
    return np.array(times), np.array(Us), pred, info


def stokes_start_time(W, reps=3):
    """Wall time of lb_stokes_start on workload W (its particles' loads drive
    the field), each repetition synchronised: (list of ms, best)."""
    lat = build_lattice(W)
    lat.sync()
    ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        lat.stokes_start()
        lat.sync()
        ms.append(1e3 * (time.perf_counter() - t0))
    del lat
    return {"workload": W.name, "storage": W.storage, "ms": [round(v, 2) for v in ms], "best_ms": round(min(ms), 2)}


def steps_to_tolerance(times, U, Uinf, tol=0.005):
    """Per particle: the first sampled step after which |U(t) - U_inf| <=
    tol |U_inf| holds until the end (inf if it never settles)."""
    dev = np.linalg.norm(U - Uinf[None], axis=2) / np.linalg.norm(Uinf, axis=1)[None]
    out = np.full(U.shape[1], np.inf)
    for i in range(U.shape[1]):
        bad = np.nonzero(dev[:, i] > tol)[0]
        if len(bad) == 0:
            out[i] = times[0]
        elif bad[-1] < len(times) - 1:
            out[i] = times[bad[-1] + 1]
    return out


def train_warm_network(seeds=4, boxes=128, epochs=600, seed0=20, storage="fp16", extra=None):
    """The warm-start network trained on the library's own ensemble runs:
    `seeds` force-driven ensembles of `boxes` boxes with config 4's
    distributions (seeds seed0, seed0 + 1, ...; every other one with
    torques), their steady samples augmented by the spheroid's symmetries and
    the linearity of Stokes flow.  extra: samples (X, Y) fed back from runs
    whose prediction missed (lb_surrogate_sample), added to the ensembles'
    before the augmentation.  Returns (surrogate, info)."""
    Xs, Ys, steps = [], [], 0
    for k in range(seeds):
        W = workloads.c4(storage, boxes, seed_index=seed0 + k, torque=(k % 2 == 0))
        X, Y, n = ensemble_samples(W, efolds=8)
        Xs.append(X)
        Ys.append(Y)
        steps += n
    if extra is not None:
        Xs.append(np.asarray(extra[0], np.float64))
        Ys.append(np.asarray(extra[1], np.float64))
    Xa, Ya = augment(np.concatenate(Xs), np.concatenate(Ys))
    sur, info = train_surrogate(Xa, Ya, epochs=epochs)
    info["lb_steps_per_ensemble"] = steps // max(seeds, 1)
    info["extra_samples"] = 0 if extra is None else len(extra[0])
    return sur, info


def watch_warm_start(W, surrogate, tol, every=25):
    """Warm-start every box of W with the surrogate, watched at tol, and step
    until every box is decided.  Returns (lattice, status per box, decision
    step per box, predictions, the particles' velocities just after each
    box's decision)."""
    lat = build_lattice(W)
    pred = lat.warm_start(surrogate, tol=tol)
    lat.set_graph(every)
    nb = len(W.boxes)
    U_dec = np.full((len(W.particles), 6), np.nan)
    decided = np.zeros(nb, dtype=bool)
    t = 0
    while not decided.all():
        lat.step(every)
        t += every
        st, at = lat.warm_status()
        new = (st >= 2) & ~decided
        if new.any():
            P = lat.particles()
            for i, p in enumerate(W.particles):
                if new[p.box]:
                    U_dec[i] = np.concatenate([P["U"][i], P["W"][i]])
            decided |= new
        assert t < 10 ** 6, "the monitor decided no box"
    st, at = lat.warm_status()
    return lat, st, at, pred, U_dec


def _body_axis(q):
    """Lab-frame body x axis of unit quaternions q (n, 4), scalar first."""
    q0, q1, q2, q3 = np.asarray(q, float).T
    return np.stack([1 - 2 * (q2 * q2 + q3 * q3), 2 * (q1 * q2 + q0 * q3), 2 * (q1 * q3 - q0 * q2)], -1)


def squirmer_starts(W, surrogate, steps=10000, every=50, monitor_tol=0.1, contact=12.0, log=None):
    """Starts of a squirmer suspension (config 5) compared through each
    swimmer's speed along its own axis, s = U . e: plain (rest), the
    surrogate warm start (its inputs the equivalent propulsive load of each
    squirmer and the box's volume per particle), the same watched by the
    device monitor at monitor_tol, and a control starting every squirmer at
    the closed-form free swimming speed (eq. squirmervel).  The paper has no
    inter-particle force: squirmers that come within `contact` of another
    centre (2a + 2 for a = 5) in any run are left out, and the latched overlap
    flags are counted.  s_inf is the plain run's mean over its last fifth;
    reported per start: the median |s - s_inf| / s_inf at sampled steps, the
    median first step at which it falls below 5% and 2%, and the fraction of
    swimmers that stay within 0.5% / 2% from some step to the end."""
    a = max(max(p.axes) for p in W.particles)
    Us = {}
    for i, p in enumerate(W.particles):
        ax = p.axes
        r = ax[0] / math.sqrt(ax[1] * ax[2])
        e = math.sqrt(1 - 1 / r ** 2) if r > 1 + 1e-6 else 0.0
        B1 = p.squirmer[0]
        Us[i] = 2 * B1 / 3 if e < 1e-3 else B1 / e * (1 / e - (1 / e ** 2 - 1) * math.atanh(e))
    runs, pos, info = {}, {}, {}
    L = np.array(W.boxes[0].shape, float)
    for start in ("plain", "surrogate", "surrogate_watched", "control"):
        lat = build_lattice(W)
        if start.startswith("surrogate"):
            pred = lat.warm_start(surrogate, tol=monitor_tol if start == "surrogate_watched" else 0.0)
            e0 = _body_axis([p.quat for p in W.particles])
            info["prediction_over_closed_form"] = float(np.median(
                (pred[:, :3] * e0).sum(1) / np.array([Us[i] for i in range(len(W.particles))])))
        elif start == "control":
            e0 = _body_axis([p.quat for p in W.particles])
            for i in range(len(W.particles)):
                lat.set_velocity(i, e0[i] * Us[i], np.zeros(3))
            lat.stokes_start()
        lat.set_graph(every)
        S, flags, X = _swim(lat, steps, every, positions=True)
        if start == "surrogate_watched":
            st, at = lat.warm_status()
            info["monitor"] = {"status": _status_name(st[0]), "decided_step": int(at[0])}
        info.setdefault("overlap_flags", {})[start] = flags
        runs[start], pos[start] = np.array(S), np.array(X)
        del lat
        if log:
            log(f"squirmer_starts: {start} run done ({steps} steps, {flags} overlap flags)")
    times = np.arange(1, steps // every + 1) * every
    close = np.zeros(len(W.particles), dtype=bool)
    for Xs in pos.values():
        for k in range(0, len(Xs), 4):
            d = Xs[k][:, None, :] - Xs[k][None, :, :]
            d -= L * np.round(d / L)
            rr = np.sqrt((d * d).sum(-1)) + 1e9 * np.eye(len(W.particles))
            close |= (rr < contact).any(1)
    keep = ~close
    tail = max(len(times) // 5, 1)
    s_inf = runs["plain"][-tail:, keep].mean(0)
    sp = runs["plain"][:, keep]
    out = {"workload": W.name, "storage": W.storage, "steps": steps, "every": every, "monitor_tol": monitor_tol,
           "swimmers": len(W.particles), "kept": int(keep.sum()), "left_out_contact": int(close.sum()),
           "plain_speed_change_over_last_2000": float(np.median(np.abs(sp[-1] - sp[-1 - 2000 // every])
                                                                / np.abs(sp[-1]))),
           "plain_speed_over_closed_form": float(np.median(sp[-1] / np.array([Us[i] for i in np.nonzero(keep)[0]]))),
           **info, "starts": {}}
    marks = [k for k in (0, 1, 3, 5, 9, 19, 39, 99, len(times) - 1) if k < len(times)]
    for start, s in runs.items():
        dev = np.abs(s[:, keep] - s_inf[None]) / np.abs(s_inf)[None]
        first = {}
        for tol in (0.05, 0.02):
            hit = dev <= tol
            idx = np.where(hit.any(0), hit.argmax(0), -1)
            first[str(tol)] = float(np.median(np.where(idx >= 0, times[np.maximum(idx, 0)], np.inf)))
        stay = {}
        for tol in (0.005, 0.02):
            stay[str(tol)] = float(np.isfinite(steps_to_tolerance(times, s[:, keep, None], s_inf[:, None], tol)).mean())
        out["starts"][start] = {"median_deviation": {int(times[k]): round(float(np.median(dev[k])), 4) for k in marks},
                                "median_first_step_within": first, "fraction_settled_to_end": stay}
    return out


def _swim(lat, steps, every, positions=False):
    """Step a squirmer lattice, counting latched overlap flags (the paper has
    no inter-particle force); returns (speeds along each swimmer's axis per
    sample, flags) and, with positions, the centres per sample as well."""
    S, X, flags = [], [], 0
    for _ in range(steps // every):
        try:
            lat.step(every)
        except lbell.LBError as err:
            if err.status != lbell.LB_EOVERLAP:
                raise
            flags += 1
        try:
            P = lat.particles()
        except lbell.LBError as err:
            if err.status != lbell.LB_EOVERLAP:
                raise
            flags += 1
            P = lat.particles()
        S.append((P["U"] * _body_axis(P["q"])).sum(1))
        if positions:
            X.append(P["x"].copy())
    return (np.array(S), flags, np.array(X)) if positions else (np.array(S), flags)


def squirmer_feedback(train, W_fit, W_eval, steps=3000, every=50, monitor_tol=0.1, log=None):
    """The learned part's loop closed on squirmer suspensions (config 5).
    train(extra) returns a network trained on the force-driven ensembles plus
    the samples `extra` (None: none).  The first network warm-starts W_fit,
    watched by the device monitor at monitor_tol; after `steps` steps the
    samples of every particle of a box the monitor flagged (fallen back or
    settled elsewhere) are fed back and the network retrained.  Both networks
    then warm-start another suspension, W_eval, watched the same way, beside
    a plain run of it: reported per network, its predicted speed along each
    swimmer's axis over the closed-form free swimming speed (eq. squirmervel)
    and over the plain run's mean over its last fifth (medians), the
    monitor's decision, the share of swimmers further than monitor_tol from
    their predictions (V = (U, a Omega), the monitor's measure) one sample
    before the decision step and their median miss, and the median
    |s - s_inf| / s_inf at a few steps."""
    def closed_form(W):
        out = []
        for p in W.particles:
            r = p.axes[0] / math.sqrt(p.axes[1] * p.axes[2])
            e = math.sqrt(1 - 1 / r ** 2) if r > 1 + 1e-6 else 0.0
            B1 = p.squirmer[0]
            out.append(2 * B1 / 3 if e < 1e-3 else B1 / e * (1 / e - (1 / e ** 2 - 1) * math.atanh(e)))
        return np.array(out)

    def watched(W, sur):
        lat = build_lattice(W)
        pred = lat.warm_start(sur, tol=monitor_tol)
        lat.set_graph(every)
        a = np.array([max(p.axes) for p in W.particles])[:, None]
        w0 = int(math.ceil(2 * a.max() ** 2 / viscosity(W)))
        before = max((w0 - 1) // every, 1) * every  # the last sample before the decision
        S1, f1 = _swim(lat, before, every)
        P = lat.particles()
        V = np.concatenate([P["U"], a * P["W"]], 1)
        Vp = np.concatenate([pred[:, :3], a * pred[:, 3:]], 1)
        miss = np.linalg.norm(V - Vp, axis=1) / np.linalg.norm(Vp, axis=1)
        S2, f2 = _swim(lat, steps - before, every)
        st, at = lat.warm_status()
        return lat, pred, np.concatenate([S1, S2]), f1 + f2, st, at, (before, miss)

    sur0 = train(None)
    lat, _, _, _, st, at, _ = watched(W_fit, sur0)
    X, Y = lat.surrogate_sample()
    del lat
    fed = np.array([i for i, p in enumerate(W_fit.particles) if st[p.box] in (3, 4)], dtype=int)
    if log:
        log(f"squirmer_feedback: fit run done, {len(fed)} samples fed back")
    sur1 = train((X[fed], Y[fed])) if len(fed) else sur0
    lat = build_lattice(W_eval)
    lat.set_graph(every)
    Sp, _ = _swim(lat, steps, every)
    del lat
    tail = max(len(Sp) // 5, 1)
    s_inf = Sp[-tail:].mean(0)
    Us = closed_form(W_eval)
    e0 = _body_axis([p.quat for p in W_eval.particles])
    times = np.arange(1, steps // every + 1) * every
    marks = [k for k in (0, 1, 5, 19, len(times) - 1) if k < len(times)]
    out = {"fit_workload": W_fit.name, "eval_workload": W_eval.name, "steps": steps, "every": every,
           "monitor_tol": monitor_tol, "fit_monitor": _status_name(st[0]), "fit_decided_step": int(at[0]),
           "samples_fed_back": int(len(fed)),
           "plain_speed_over_closed_form": round(float(np.median(s_inf / Us)), 4), "networks": {}}
    for name, sur in (("before_feedback", sur0), ("after_feedback", sur1)):
        lat, pred, S, flags, st, at, (t_miss, miss) = watched(W_eval, sur)
        del lat
        sp = (pred[:, :3] * e0).sum(1)
        dev = np.abs(S - s_inf[None]) / np.abs(s_inf)[None]
        out["networks"][name] = {
            "prediction_over_closed_form": round(float(np.median(sp / Us)), 4),
            "prediction_over_plain": round(float(np.median(sp / s_inf)), 4),
            "monitor": _status_name(st[0]), "decided_step": int(at[0]), "overlap_flags": flags,
            "miss_step": t_miss, "share_missing": round(float((miss > monitor_tol).mean()), 4),
            "median_miss": round(float(np.median(miss)), 4),
            "median_deviation": {int(times[k]): round(float(np.median(dev[k])), 4) for k in marks}}
        if log:
            log(f"squirmer_feedback: {name} run done")
    return out


def _status_name(code):
    return lbell.Lattice.WARM_STATUS[int(code)]


def compare_starts(W, surrogate, efolds=12.0, every=25, tol=0.005, monitor_tol=0.1):
    """Steps to a tol-accurate steady velocity for each particle of the
    force-driven ensemble W from the three starts, and from the start field
    with the exact steady velocities (the field's own share).  The steady
    velocity is the end of the plain run; a box counts only if that run
    changed by less than 0.05% over its last slow time.  The surrogate run is watched on the
    device (lb_warm_start with monitor_tol): at W0 = ceil(2 a^2 / nu) steps a
    box whose velocity missed the prediction while the run still moved falls
    back to the plain start, and its steps count from the warm start; boxes
    that missed, fell back or not, have their samples (at the end of the run)
    queued for training."""
    nu = viscosity(W)
    steps = int(math.ceil(efolds * max(slow_time(box_edge(W, i), nu) for i in range(len(W.particles)))))
    steps = (steps + every - 1) // every * every
    tp, Up, _, _ = trajectory(W, "plain", steps=steps, every=every)
    ts, Us, pred, info = trajectory(W, "surrogate", surrogate, steps=steps, every=every, tol=monitor_tol)
    tc, Uc, _, cinfo = trajectory(W, "control", steps=steps, every=every)
    Uinf = Up[-1]
    tx, Ux, _, _ = trajectory(W, "given", steps=steps, every=every, velocities=Uinf)
    ok = np.ones(len(W.particles), dtype=bool)
    for i, p in enumerate(W.particles):
        lag = int(round(slow_time(box_edge(W, i), nu) / every))
        ok[i] = np.linalg.norm(Up[-1, i] - Up[-1 - lag, i]) < 5e-4 * np.linalg.norm(Uinf[i])
    status = np.array([info["status"][p.box] for p in W.particles])
    n = {"plain": steps_to_tolerance(tp, Up, Uinf, tol), "surrogate": steps_to_tolerance(ts, Us, Uinf, tol),
         "control": steps_to_tolerance(tc, Uc, Uinf, tol), "exact_velocity": steps_to_tolerance(tx, Ux, Uinf, tol)}
    err0 = {"surrogate": np.linalg.norm(Us[0] - Uinf, axis=1) / np.linalg.norm(Uinf, axis=1),
            "control": np.linalg.norm(Uc[0] - Uinf, axis=1) / np.linalg.norm(Uinf, axis=1)}
    pred_err = np.linalg.norm(pred[:, :3] - Uinf, axis=1) / np.linalg.norm(Uinf, axis=1)
    med = {k: float(np.median(v[ok])) if ok.any() else float("nan") for k, v in n.items()}
    rate = lambda code: float((status[ok] == code).mean()) if ok.any() else float("nan")  # noqa: E731
    queued = np.nonzero(ok & ((status == 3) | (status == 4)))[0]
    X, Y = info["samples"]
    return {"boxes": int(len(W.particles)), "steady_boxes": int(ok.sum()), "steps": steps, "every": every,
            "tol": tol, "monitor_tol": monitor_tol, "median_steps": med,
            "surrogate_over_plain": med["surrogate"] / med["plain"],
            "control_over_plain": med["control"] / med["plain"],
            "median_prediction_error": float(np.median(pred_err[ok])) if ok.any() else float("nan"),
            "median_error_after_first_sample": {k: float(np.median(v[ok])) if ok.any() else float("nan")
                                                for k, v in err0.items()},
            "accepted_rate": rate(2), "fallback_rate": rate(3), "steady_miss_rate": rate(4),
            "median_steps_fallback_boxes": (float(np.median(n["surrogate"][ok & (status == 3)]))
                                            if (ok & (status == 3)).any() else None),
            "median_steps_plain_fallback_boxes": (float(np.median(n["plain"][ok & (status == 3)]))
                                                  if (ok & (status == 3)).any() else None),
            "median_decision_step_fallback_boxes": (float(np.median(np.array(
                [info["decided"][p.box] for p in W.particles])[ok & (status == 3)]))
                if (ok & (status == 3)).any() else None),
            "queued": queued.tolist(), "queued_samples": (X[queued], Y[queued]),
            "start_ms": {"surrogate": info["start_ms"], "control": cinfo["start_ms"]},
            "per_box": n, "steady": ok, "status": status}
