"""FP64 reference of the learned warm start: the MLP surrogate (forward,
backward, Adam), its input features and output scaling, the Stokes start
field, and the unbounded-fluid closed forms used as a control.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``; never by the product
path.  Plain numpy in float64, written from the definitions; it shares no
code with the HIP library.

Definitions (the paper has no learned part; the surrogate is specified by the
task, and the readings are listed with the design notes):

* network 8 -> 64 -> 64 -> 6, tanh hidden layers, linear output;
  parameters flat, in the order W1[64][8], b1[64], W2[64][64], b2[64],
  W3[6][64], b3[6] (5126 values);
* loss: mean squared error over the n x 6 outputs;
* Adam (Kingma & Ba 2015): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected;
* BF16 mode: the operands of every matrix product (inputs, weights, hidden
  activations, back-propagated errors) are rounded to bfloat16 (round to
  nearest even) at the points where the GPU kernels round them; sums, biases,
  tanh and the error terms stay in full precision.
"""
import math

import numpy as np

N_IN, N_H, N_OUT = 8, 64, 6
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


# ------------------------------------------------------------------ bfloat16 --

def bf16(x):
    """Round float32 values of x to bfloat16 (nearest, ties to even); returns float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    r = np.where(nan, u, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- parameters --

def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == N_PARAMS
    out, k = {}, 0
    for name, s in SHAPES:
        n = int(np.prod(s))
        out[name] = p[k:k + n].reshape(s)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


# -------------------------------------------------------------------- network --

def forward(p, X, bf=False):
    """Outputs (n, 6) and the cache of activations."""
    P = unpack(p)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    h1 = np.tanh(x @ W1.T + P["b1"])
    h1r = r(h1)
    h2 = np.tanh(h1r @ W2.T + P["b2"])
    h2r = r(h2)
    y = h2r @ W3.T + P["b3"]
    return y, {"x": x, "h1": h1r, "h2": h2r, "W1": W1, "W2": W2, "W3": W3}


def loss_grad(p, X, Y, bf=False):
    """Mean squared error over all outputs and its gradient (flat, like p)."""
    X, Y = np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64)
    n = X.shape[0]
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(p, X, bf)
    L = float(np.sum((y - Y) ** 2) / (n * N_OUT))
    d3 = 2.0 * (y - Y) / (n * N_OUT)               # dL/dy
    d3r = r(d3)
    g = {"W3": d3r.T @ c["h2"], "b3": d3.sum(0)}
    d2 = (d3r @ c["W3"]) * (1.0 - c["h2"] ** 2)     # dL/d(pre-activation of layer 2)
    d2r = r(d2)
    g["W2"], g["b2"] = d2r.T @ c["h1"], d2.sum(0)
    d1 = (d2r @ c["W2"]) * (1.0 - c["h1"] ** 2)
    d1r = r(d1)
    g["W1"], g["b1"] = d1r.T @ c["x"], d1.sum(0)
    return L, pack(g)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------ features and scaling --

def rotmat(q):
    """Body -> lab rotation of the unit quaternion (scalar first)."""
    q0, q1, q2, q3 = [float(v) for v in q]
    return np.array([[1 - 2 * (q2 * q2 + q3 * q3), 2 * (q1 * q2 - q0 * q3), 2 * (q1 * q3 + q0 * q2)],
                     [2 * (q1 * q2 + q0 * q3), 1 - 2 * (q1 * q1 + q3 * q3), 2 * (q2 * q3 - q0 * q1)],
                     [2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1), 1 - 2 * (q1 * q1 + q2 * q2)]])


def req(axes):
    """Radius of the sphere of equal volume."""
    a, b, c = axes
    return (a * b * c) ** (1.0 / 3.0)


def features(axes, q, F, T, box, n_box=1, B1=0.0, mu=1.0):
    """Input vector (ln r, a/L, F_body/s, T_body/(R s)), with r = a/sqrt(bc),
    L = cube root of the box volume per particle (n_box particles in the
    box), R the equal-volume radius and s = sqrt(|F|^2 + (|T|/R)^2); zero
    load gives zero load components.  A squirmer (B1 != 0) adds its
    equivalent propulsive force (propulsive_force) along body x to F_body."""
    a, b, c = axes
    R = req(axes)
    L = (box[0] * box[1] * box[2] / n_box) ** (1.0 / 3.0)
    Rm = rotmat(q)
    Fb, Tb = Rm.T @ np.asarray(F, float), Rm.T @ np.asarray(T, float)
    Fb[0] += propulsive_force(axes, B1, mu)
    s = math.sqrt(Fb @ Fb + (Tb @ Tb) / (R * R))
    x = np.zeros(8)
    x[0] = math.log(a / math.sqrt(b * c))
    x[1] = a / L
    if s > 0:
        x[2:5] = Fb / s
        x[5:8] = Tb / (R * s)
    return x, s


def velocities(y, axes, q, F, T, nu, rho0=1.0, B1=0.0):
    """Lab-frame (U, Omega) from the network output y (normalised body-frame
    response): U_body = y[0:3] s / (6 pi mu R), Omega_body = y[3:6] s / (8 pi mu R^2)."""
    R = req(axes)
    mu = rho0 * nu
    _, s = features(axes, q, F, T, (1, 1, 1), B1=B1, mu=mu)
    Rm = rotmat(q)
    Ub = np.asarray(y[0:3], float) * s / (6 * math.pi * mu * R)
    Wb = np.asarray(y[3:6], float) * s / (8 * math.pi * mu * R * R)
    return Rm @ Ub, Rm @ Wb


def targets(U, W, axes, q, F, T, nu, rho0=1.0, B1=0.0):
    """Inverse of velocities(): the normalised output for measured (U, Omega)."""
    R = req(axes)
    mu = rho0 * nu
    _, s = features(axes, q, F, T, (1, 1, 1), B1=B1, mu=mu)
    Rm = rotmat(q)
    y = np.zeros(6)
    y[0:3] = Rm.T @ np.asarray(U, float) * 6 * math.pi * mu * R / s
    y[3:6] = Rm.T @ np.asarray(W, float) * 8 * math.pi * mu * R * R / s
    return y


# --------------------------------------------------------- Stokes start field --

def equilibrium(rho, u):
    """Second-order D3Q19 equilibria for velocities u (n, 3) -> (n, 19), in the
    direction order rest, +-x, +-y, +-z, then (1,1,0), (-1,-1,0), (1,-1,0),
    (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1),
    (0,1,-1), (0,-1,1)."""
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                  [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    u = np.atleast_2d(u)
    cu = u @ c.T
    uu = (u * u).sum(1, keepdims=True)
    return rho * w * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def min_image(d, n):
    d = np.array(d, dtype=float)
    for k in range(3):
        d[..., k] = np.where(d[..., k] >= n[k] / 2, d[..., k] - n[k], d[..., k])
        d[..., k] = np.where(d[..., k] < -n[k] / 2, d[..., k] + n[k], d[..., k])
    return d


def stokes_velocity(d, U, W, R):
    """Creeping flow around a sphere of radius R translating with U and
    rotating with W, at offsets d (n, 3) from its centre: the Stokes solution
    u = (3R/4r)(U + (U.e)e) + (R^3/4r^3)(U - 3(U.e)e) plus the rotlet
    (R/r)^3 W x d outside, rigid motion U + W x d inside."""
    d = np.atleast_2d(d)
    r = np.linalg.norm(d, axis=1)[:, None]
    U, W = np.asarray(U, float), np.asarray(W, float)
    rigid = U + np.cross(W, d)
    rs = np.maximum(r, 1e-300)
    e = d / rs
    Ue = (e @ U)[:, None]
    out = (3 * R / (4 * rs)) * (U + Ue * e) + (R ** 3 / (4 * rs ** 3)) * (U - 3 * Ue * e) \
        + (R / rs) ** 3 * np.cross(W, d)
    return np.where(r >= R, out, rigid)


# Below this eccentricity a prolate spheroid's flow is taken as the sphere's
# (they differ by O(e^2)).
E_LINE = 1e-4


def _gl_panels(x0, delta, lo, hi, npt=16, ratio=2.0):
    """Nodes and weights of a composite Gauss-Legendre rule on [lo, hi]
    (lo <= x0 <= hi) whose panels grow geometrically away from x0: panel j
    on each side spans distances delta (ratio^j - 1) .. delta (ratio^(j+1) -
    1) from x0, clipped to the interval.  Arrays over leading dimensions of
    x0 / delta; returns (xi, w) with a trailing node axis."""
    t, wt = np.polynomial.legendre.leggauss(npt)
    span = np.maximum(np.max(np.maximum(x0 - lo, hi - x0) / delta), 1.0)
    J = int(math.ceil(math.log(1.0 + span) / math.log(ratio))) + 1
    xs, ws = [], []
    for j in range(J):
        d0, d1 = delta * (ratio ** j - 1.0), delta * (ratio ** (j + 1) - 1.0)
        for sgn, end in ((-1.0, lo), (1.0, hi)):
            room = np.abs(end - x0)
            a, b = np.minimum(d0, room), np.minimum(d1, room)
            half, mid = 0.5 * (b - a), 0.5 * (b + a)
            xs.append(x0[..., None] + sgn * (mid[..., None] + half[..., None] * t))
            ws.append(half[..., None] * wt)
    return np.concatenate(xs, axis=-1), np.concatenate(ws, axis=-1)


def spheroid_flow(d, axes, q, F, T, mu):
    """Creeping flow of an unbounded fluid around a rigid prolate spheroid
    (semi-axes a > b = c, orientation q) under the load (F, T), at offsets
    d (n, 3) from its centre; rigid motion inside.

    The body moves with the velocities of the resistance functions
    (unbounded_velocities).  Outside, the flow is that of singularities on
    the focal segment |xi| <= f = a e of the axis p (Chwang & Wu, J. Fluid
    Mech. 63, 1974, and 67, 1975), with g = f^2 - xi^2, r = d - xi p, R = |r|,
    s = F / (16 pi mu f), t = T / (8 pi mu (4/3) f^3), t_c the part of t
    across p and m = t_c x p:
      Stokeslets            s / R + (s.r) r / R^3,
      potential dipoles     -(1 - e^2) / (2 e^2) g (-s / R^3 + 3 (s.r) r / R^5),
      rotlets               g t x r / R^3,
      stresslets            3 e^2 / (2 - e^2) g r (r.p)(r.m) / R^5,
      potential quadrupoles (1 - e^2) / (4 (2 - e^2)) g^2 (p.grad_r) of the
                            dipole -m / R^3 + 3 (m.r) r / R^5,
    integrated over xi by composite Gauss-Legendre quadrature on panels that
    grow geometrically from the point of the segment nearest d."""
    d = np.atleast_2d(np.asarray(d, float))
    a, b, _ = axes
    e2 = 1.0 - (b / a) ** 2
    e = math.sqrt(e2)
    f = a * e
    U, W = unbounded_velocities(axes, q, F, T, mu)
    p = rotmat(q)[:, 0]
    F, T = np.asarray(F, float), np.asarray(T, float)
    s = F / (16 * math.pi * mu * f)
    t = T / (8 * math.pi * mu * 4.0 / 3.0 * f ** 3)
    m = np.cross(t - (t @ p) * p, p)
    z = d @ p
    rho2 = np.maximum((d * d).sum(1) - z * z, 0.0)
    inside = z * z / (a * a) + rho2 / (b * b) < 1.0
    x0 = np.clip(z, -f, f)
    delta = np.sqrt(rho2 + (z - x0) ** 2)
    out = U + np.cross(W, d)
    o = ~inside
    if o.any():
        xi, w = _gl_panels(x0[o], delta[o], -f, f)
        r = d[o][:, None, :] - xi[..., None] * p                      # (n, k, 3)
        R = np.sqrt((r * r).sum(-1))[..., None]
        g = (f * f - xi * xi)[..., None]
        rp = (r @ p)[..., None]
        rm = (r @ m)[..., None]
        sr = (r @ s)[..., None]
        val = (s / R + sr * r / R ** 3
               - (1 - e2) / (2 * e2) * g * (-s / R ** 3 + 3 * sr * r / R ** 5)
               + g * np.cross(t, r) / R ** 3
               + 3 * e2 / (2 - e2) * g * r * rp * rm / R ** 5
               + (1 - e2) / (4 * (2 - e2)) * g * g * (3 * (m * rp + rm * p) / R ** 5 - 15 * rm * rp * r / R ** 7))
        out[o] = (w[..., None] * val).sum(1)
    return out


def spheroid_pressure(d, axes, q, F, T, mu):
    """Pressure of spheroid_flow at offsets d (n, 3): that of its Stokeslets,
    2 mu (s.r) / R^3, and of its stresslets, 3 e^2 / (2 - e^2) g
    2 mu (r.p)(r.m) / R^5, integrated over the focal segment (the potential
    dipoles and quadrupoles and the rotlets carry none); 0 inside the body."""
    d = np.atleast_2d(np.asarray(d, float))
    a, b, _ = axes
    e2 = 1.0 - (b / a) ** 2
    f = a * math.sqrt(e2)
    p = rotmat(q)[:, 0]
    F, T = np.asarray(F, float), np.asarray(T, float)
    s = F / (16 * math.pi * mu * f)
    t = T / (8 * math.pi * mu * 4.0 / 3.0 * f ** 3)
    m = np.cross(t - (t @ p) * p, p)
    z = d @ p
    rho2 = np.maximum((d * d).sum(1) - z * z, 0.0)
    inside = z * z / (a * a) + rho2 / (b * b) < 1.0
    x0 = np.clip(z, -f, f)
    delta = np.sqrt(rho2 + (z - x0) ** 2)
    out = np.zeros(len(d))
    o = ~inside
    if o.any():
        xi, w = _gl_panels(x0[o], delta[o], -f, f)
        r = d[o][:, None, :] - xi[..., None] * p
        R = np.sqrt((r * r).sum(-1))
        g = f * f - xi * xi
        val = 2 * mu * ((r @ s) / R ** 3 + 3 * e2 / (2 - e2) * g * (r @ p) * (r @ m) / R ** 5)
        out[o] = (w * val).sum(1)
    return out


def particle_pressure(d, p, mu):
    """Pressure of particle_flow at offsets d: spheroid_pressure, or for the
    sphere of radius R the Stokes solution's 3 mu R (U.d) / (2 r^3) =
    F.d / (4 pi r^3) outside R (the rotlet carries none); 0 inside."""
    a, b, c = p["axes"]
    F, T = np.asarray(p["F"], float), np.asarray(p["T"], float)
    if a > b and b == c and 1.0 - (b / a) ** 2 >= E_LINE ** 2:
        return spheroid_pressure(d, p["axes"], p["q"], F, T, mu)
    d = np.atleast_2d(np.asarray(d, float))
    R = req(p["axes"])
    r = np.linalg.norm(d, axis=1)
    return np.where(r >= R, (d @ F) / (4 * math.pi * np.maximum(r, 1e-300) ** 3), 0.0)


def particle_flow(d, p, mu):
    """Free-space flow that particle p (dict: axes, q, F, T) drives at
    offsets d: spheroid_flow for a prolate spheroid (a > b = c, eccentricity
    at least E_LINE); otherwise the sphere of the equal-volume radius R moving
    with F / (6 pi mu R) and turning with T / (8 pi mu R^3) (stokes_velocity)."""
    a, b, c = p["axes"]
    F, T = np.asarray(p["F"], float), np.asarray(p["T"], float)
    if a > b and b == c and 1.0 - (b / a) ** 2 >= E_LINE ** 2:
        return spheroid_flow(d, p["axes"], p["q"], F, T, mu)
    R = req(p["axes"])
    return stokes_velocity(d, F / (6 * math.pi * mu * R), T / (8 * math.pi * mu * R ** 3), R)


KMAX = 2  # Fourier modes |n_i| <= KMAX of the box carry the periodic correction


def _is_line(axes):
    """A prolate spheroid a > b = c of eccentricity at least E_LINE."""
    if axes is None:
        return False
    a, b, c = axes
    return a > b and b == c and 1.0 - (b / a) ** 2 >= E_LINE ** 2


def rotation_traction(k, T, R, axes=None, q=None):
    """Transform of the traction a torque T spreads over a body, f_hat(k) =
    -3 i (Q^T k) j1(kappa) / kappa, at wave vectors k (m, 3).  The traction
    of a body in rigid motion is sigma(x) C x, sigma the uniform layer of the
    unit sphere mapped onto the surface and C constant, so its transform is
    C (i grad_k) sinc(kappa) with C = 3 Q^T A^-2, Q = integral of x f^T its
    first moment: the torque's antisymmetric part Q_kj = eps_kji T_i / 2, and
    for a prolate spheroid (axis p, eccentricity e) the stresslet of its
    line solution (spheroid_flow), e^2 / (2 - e^2) sym(p (T_c x p)), T_c the
    torque across p, kappa = |diag(a, b, c) R(q)^T k|; any other body is
    taken as the sphere of radius R (kappa = |k| R, no stresslet).  Returns
    (Q^T k, j1(kappa) / kappa)."""
    k = np.atleast_2d(np.asarray(k, float))
    T = np.asarray(T, float)
    g = -0.5 * np.cross(k, T)              # Q_A^T k
    if _is_line(axes):
        a, b, _ = axes
        e2 = 1.0 - (b / a) ** 2
        p = rotmat(q)[:, 0]
        m = np.cross(T - (T @ p) * p, p)
        cs = e2 / (2 - e2) / 2
        g = g + cs * (np.outer(k @ m, p) + np.outer(k @ p, m))   # + Q_S k
        kap = np.linalg.norm((k @ rotmat(q)) * np.asarray(axes, float), axis=1)
    else:
        kap = np.sqrt((k * k).sum(1)) * R
    return g, (np.sin(kap) - kap * np.cos(kap)) / kap ** 3


def periodic_modes(k, F, T, R, mu, V, axes=None, q=None):
    """Fourier coefficients (1/V) u_hat(k) of the creeping flow driven by a
    force F and a torque T spread over a sphere of radius R (uniform surface
    traction), at wave vectors k (m, 3), none zero, for a periodic box of
    volume V, centre at the origin:
      u_hat = (I - k k / k^2) f_hat / (mu k^2),
      f_hat = F sinc(kR) + i (k x T) 3 j1(kR) / (2 kR).
    With the semi-axes and orientation of an ellipsoid, the force is spread
    as the traction on that ellipsoid translating (the sphere's uniform layer
    mapped by diag(a, b, c) in the body frame), whose transform is
    sinc(|diag(a, b, c) R(q)^T k|), and the torque as rotation_traction (the
    rotating prolate spheroid's, the sphere's otherwise)."""
    k = np.atleast_2d(np.asarray(k, float))
    F, T = np.asarray(F, float), np.asarray(T, float)
    k2 = (k * k).sum(1)
    x = np.sqrt(k2) * R
    if axes is None:
        sinc = np.sin(x) / x
    else:
        xa = np.linalg.norm((k @ rotmat(q)) * np.asarray(axes, float), axis=1)
        sinc = np.sin(xa) / xa
    g, j1k = rotation_traction(k, T, R, axes, q)
    f = F[None, :] * sinc[:, None] - 3j * g * j1k[:, None]
    Pf = f - k * ((k * f).sum(1) / k2)[:, None]
    return Pf / (mu * k2)[:, None] / V


def periodic_pressure_modes(k, F, R, V, axes=None, q=None, T=None):
    """Fourier coefficients (1/V) p_hat(k) of the pressure of the periodic
    flow of periodic_modes: from mu k^2 u_hat = f_hat - i k p_hat with
    k.u_hat = 0, p_hat = -i (k.f_hat) / k^2, f_hat the spread force and
    torque (the torque's antisymmetric part has no divergence and drives
    none; a prolate spheroid's stresslet does)."""
    k = np.atleast_2d(np.asarray(k, float))
    F = np.asarray(F, float)
    k2 = (k * k).sum(1)
    if axes is None:
        xa = np.sqrt(k2) * R
    else:
        xa = np.linalg.norm((k @ rotmat(q)) * np.asarray(axes, float), axis=1)
    f = F[None, :] * (np.sin(xa) / xa)[:, None]
    if T is not None:
        g, j1k = rotation_traction(k, T, R, axes, q)
        f = f - 3j * g * j1k[:, None]
    return -1j * (k * f).sum(1) / k2 / V


def periodic_coefficients(shape, centre, F, T, R, mu, axes=None, q=None, pressure=False):
    """Low-mode content (|n_i| <= KMAX, n != 0; fewer along an axis shorter
    than 2 KMAX + 1) of the periodic flow of a particle at `centre`:
    periodic_modes at k = 2 pi n / L times exp(-i k . x_c).  Returns (list of
    n, complex array (len, 3)); with pressure=True those of the pressure
    (periodic_pressure_modes), complex array (len,)."""
    L = np.asarray(shape, float)
    K = [min(KMAX, (int(l) - 1) // 2) for l in shape]
    ns = [(nx, ny, nz) for nz in range(-K[2], K[2] + 1) for ny in range(-K[1], K[1] + 1)
          for nx in range(-K[0], K[0] + 1) if (nx, ny, nz) != (0, 0, 0)]
    k = 2 * np.pi * np.array(ns, float) / L
    ph = np.exp(-1j * (k @ np.asarray(centre, float)))
    if pressure:
        return ns, periodic_pressure_modes(k, F, R, float(np.prod(L)), axes, q, T) * ph
    c = periodic_modes(k, F, T, R, mu, float(np.prod(L)), axes, q)
    return ns, c * ph[:, None]


def free_field(shape, particles, mu, pressure=False):
    """Sum over the particles of the free-space flow their loads drive
    (particle_flow), at minimum-image offsets; with pressure=True also its
    pressure (particle_pressure): (pos, u, p)."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(float)
    u = np.zeros((pos.shape[0], 3))
    for p in particles:
        d = min_image(pos - np.asarray(p["centre"], float), shape)
        u += particle_flow(d, p, mu)
    if not pressure:
        return pos, u
    pr = np.zeros(pos.shape[0])
    for p in particles:
        pr += particle_pressure(min_image(pos - np.asarray(p["centre"], float), shape), p, mu)
    return pos, u, pr


def start_state(shape, owner, particles, mu):
    """Density and velocity of every node of a periodic box for the warm
    start: (rho (N,), u (N, 3)).

    particles: list of dicts (centre, axes, q, F, T: the external load, U, W:
    the particle's velocities, M).  The fluid's velocity and pressure are the
    free-space flow of every particle's load and its pressure (free_field)
    whose Fourier modes |n_i| <= KMAX are replaced by those of the periodic
    solution (periodic_coefficients), so the slow modes of the box start at
    their steady values; the DFT is over all nodes (numpy's FFT).  A fluid
    node (owner 0) gets the density rho = 1 + 3 (p - pbar) (p = c_s^2
    (rho - rho0), rho0 = 1, pbar the mean over the fluid nodes: the fluid's
    mass is unchanged) and loses the uniform velocity
    ubar = (sum rho u + sum M U) / N_fluid that makes the total momentum
    (fluid sum rho u plus particles M U) zero; nodes of particle p have
    rho = 1 and move rigidly with its U, W."""
    nx, ny, nz = shape
    pos, u, pr = free_field(shape, particles, mu, pressure=True)
    N = nx * ny * nz
    L = np.asarray(shape, float)
    Su = np.fft.fftn(u.reshape(nz, ny, nx, 3), axes=(0, 1, 2))   # sum_x u exp(-2 pi i n . x / L)
    Sp = np.fft.fftn(pr.reshape(nz, ny, nx))
    cu = np.zeros((N, 3), dtype=complex)
    cp = np.zeros(N, dtype=complex)
    for p in particles:
        args = (shape, p["centre"], p["F"], p["T"], req(p["axes"]), mu, p["axes"], p["q"])
        ns, c = periodic_coefficients(*args)
        _, c_p = periodic_coefficients(*args, pressure=True)
        for n, cn, pn in zip(ns, c, c_p):
            ph = np.exp(2j * np.pi * (pos @ (np.asarray(n, float) / L)))
            cu += cn[None, :] * ph[:, None]
            cp += pn * ph
    ns, _ = periodic_coefficients(shape, (0, 0, 0), (0, 0, 0), (0, 0, 0), 1.0, 1.0)
    for n in ns:
        ph = np.exp(2j * np.pi * (pos @ (np.asarray(n, float) / L)))
        cu -= (Su[n[2] % nz, n[1] % ny, n[0] % nx] / N)[None, :] * ph[:, None]
        cp -= Sp[n[2] % nz, n[1] % ny, n[0] % nx] / N * ph
    u = u + cu.real
    pr = pr + cp.real
    owner = np.asarray(owner).ravel()
    fluid = owner == 0
    rho = np.ones(N)
    P = np.zeros(3)
    for k, p in enumerate(particles):
        mine = owner == k + 1
        d = min_image(pos[mine] - np.asarray(p["centre"], float), shape)
        u[mine] = np.asarray(p["U"], float) + np.cross(np.asarray(p["W"], float), d)
        P += p["M"] * np.asarray(p["U"], float)
    rho[fluid] = 1.0 + 3.0 * (pr[fluid] - pr[fluid].mean())
    ubar = ((rho[fluid, None] * u[fluid]).sum(0) + P) / fluid.sum()
    u[fluid] -= ubar
    return rho, u


def start_field(shape, owner, particles, mu):
    """The velocity of start_state."""
    return start_state(shape, owner, particles, mu)[1]


# ----------------------------------------------- unbounded-fluid closed forms --

def kim_karrila(r):
    """Resistance functions of a prolate spheroid with aspect ratio r >= 1
    (Kim & Karrila, Microhydrodynamics, Table 3.4): X^A, Y^A (translation
    along / across the axis, force 6 pi mu a X U) and X^C, Y^C (rotation
    about / across the axis, torque 8 pi mu a^3 X Omega); all 1 for a sphere."""
    if r < 1 + 1e-6:
        return 1.0, 1.0, 1.0, 1.0
    e = math.sqrt(1 - 1 / r ** 2)
    Lg = math.log((1 + e) / (1 - e))
    XA = 8 / 3 * e ** 3 / (-2 * e + (1 + e * e) * Lg)
    YA = 16 / 3 * e ** 3 / (2 * e + (3 * e * e - 1) * Lg)
    XC = 4 / 3 * e ** 3 * (1 - e * e) / (2 * e - (1 - e * e) * Lg)
    YC = 4 / 3 * e ** 3 * (2 - e * e) / (-2 * e + (1 + e * e) * Lg)
    return XA, YA, XC, YC


def squirmer_speed(r, B1):
    """Free swimming speed of a prolate spheroidal squirmer of aspect ratio
    r >= 1 with first slip mode B1 (Sec. III.D, eq. squirmervel; Keller & Wu
    1977): U_s = B1 e^-1 (e^-1 - (e^-2 - 1) arcoth(1/e)), e the
    eccentricity; 2 B1 / 3 for a sphere."""
    if r < 1 + 1e-6:
        return 2.0 * B1 / 3.0
    e = math.sqrt(1 - 1 / r ** 2)
    return B1 / e * (1 / e - (1 / e ** 2 - 1) * math.atanh(e))


def propulsive_force(axes, B1, mu):
    """Equivalent propulsive load of a squirmer with semi-axes (a, b, c),
    a >= b = c: the drag 6 pi mu a X^A U_s of the spheroid translating along
    its axis at its free swimming speed; 0 for B1 = 0."""
    if B1 == 0.0:
        return 0.0
    a, b, c = axes
    r = a / math.sqrt(b * c)
    return 6 * math.pi * mu * a * kim_karrila(r)[0] * squirmer_speed(r, B1)


def unbounded_velocities(axes, q, F, T, nu, rho0=1.0):
    """Velocities of a prolate spheroid (a, b, b), a >= b, under (F, T) in an
    unbounded fluid, from the resistance functions."""
    a, b, _ = axes
    XA, YA, XC, YC = kim_karrila(a / b)
    mu = rho0 * nu
    Rm = rotmat(q)
    Fb, Tb = Rm.T @ np.asarray(F, float), Rm.T @ np.asarray(T, float)
    Ub = np.array([Fb[0] / XA, Fb[1] / YA, Fb[2] / YA]) / (6 * math.pi * mu * a)
    Wb = np.array([Tb[0] / XC, Tb[1] / YC, Tb[2] / YC]) / (8 * math.pi * mu * a ** 3)
    return Rm @ Ub, Rm @ Wb
