"""Pins of the surrogate reference (oracle/surrogate.py) against what fixes
it independently of itself: finite differences and torch autograd for the
network gradient, torch's bfloat16 conversion, Adam's closed-form first
step, frame and scale invariances of the features, exact properties of the
Stokes solution, and Perrin's independent formulas for the spheroid
resistance functions."""
import math

import numpy as np
import pytest

from oracle import surrogate as S
from paper_2403_05443_amd import workloads


def _rand_params(seed, scale=0.5):
    g = np.random.default_rng(seed)
    return g.uniform(-scale, scale, S.N_PARAMS)


def _rand_data(seed, n=13):
    g = np.random.default_rng(seed)
    return g.uniform(-1, 1, (n, 8)), g.uniform(-1, 1, (n, 6))


def test_parameter_count():
    assert S.N_PARAMS == 5126
    p = np.arange(S.N_PARAMS, dtype=float)
    assert np.array_equal(S.pack(S.unpack(p)), p)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(3)
    x = np.concatenate([g.standard_normal(5000).astype(np.float32) * 10.0 ** g.integers(-8, 8, 5000),
                        np.float32([1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, -0.0, 65504.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)
    # ties to even at 1: spacing 2^-7
    assert S.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert S.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_forward_matches_torch():
    torch = pytest.importorskip("torch")
    p, (X, Y) = _rand_params(1), _rand_data(2)
    P = {k: torch.tensor(v) for k, v in S.unpack(p).items()}
    Xt = torch.tensor(X)
    h1 = torch.tanh(torch.nn.functional.linear(Xt, P["W1"], P["b1"]))
    h2 = torch.tanh(torch.nn.functional.linear(h1, P["W2"], P["b2"]))
    y = torch.nn.functional.linear(h2, P["W3"], P["b3"])
    assert np.allclose(S.forward(p, X)[0], y.numpy(), rtol=0, atol=1e-14)


def test_gradient_matches_autograd():
    torch = pytest.importorskip("torch")
    p, (X, Y) = _rand_params(4), _rand_data(5)
    pt = torch.tensor(p, requires_grad=True)
    sizes = [int(np.prod(s)) for _, s in S.SHAPES]
    parts = torch.split(pt, sizes)
    W1, b1, W2, b2, W3, b3 = [t.reshape(s) for t, (_, s) in zip(parts, S.SHAPES)]
    Xt, Yt = torch.tensor(X), torch.tensor(Y)
    h1 = torch.tanh(Xt @ W1.T + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    L = ((h2 @ W3.T + b3 - Yt) ** 2).mean()
    L.backward()
    L0, g = S.loss_grad(p, X, Y)
    assert abs(L0 - L.item()) < 1e-14
    assert np.abs(g - pt.grad.numpy()).max() <= 1e-13 * np.abs(g).max()


def test_gradient_central_differences():
    """Every one of the 5126 partial derivatives against a central difference
    with h = 1e-6: relative error below 1e-7 of the gradient's scale."""
    p, (X, Y) = _rand_params(6), _rand_data(7, n=9)
    _, g = S.loss_grad(p, X, Y)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(S.N_PARAMS):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (S.loss_grad(p + e, X, Y)[0] - S.loss_grad(p - e, X, Y)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * np.abs(g).max()


def test_bf16_mode_is_close_to_exact():
    """Rounding the product operands to bfloat16 (8 significant bits) moves
    the loss and the gradient by no more than a few ulps of bfloat16."""
    p, (X, Y) = _rand_params(8), _rand_data(9, n=64)
    L, g = S.loss_grad(p, X, Y)
    Lb, gb = S.loss_grad(p, X, Y, bf=True)
    assert abs(Lb - L) < 3 * 2 ** -8 * L
    assert np.abs(gb - g).max() < 6 * 2 ** -8 * np.abs(g).max()
    assert not np.array_equal(gb, g)


def test_bf16_mode_equals_exact_on_representable_network():
    """With bfloat16-exact inputs and weights and a network whose hidden
    activations are exactly 0 (zero first-layer weights and biases) the two
    modes agree to rounding of the sums."""
    p = S.unpack(S.bf16(_rand_params(10)))
    p["W1"][:] = 0
    p["b1"][:] = 0
    p["W2"][:] = 0
    p["b2"][:] = 0
    q = S.pack(p)
    X, Y = _rand_data(11)
    X = S.bf16(X)
    y0, _ = S.forward(q, X)
    y1, _ = S.forward(q, X, bf=True)
    assert np.allclose(y0, np.broadcast_to(p["b3"], y0.shape), atol=0)
    assert np.array_equal(y0, y1)


def test_adam_first_step_closed_form():
    """From zero moments the first bias-corrected step is lr g / (|g| + eps)."""
    g = np.array([3.0, -1e-3, 0.5, 0.0])
    p = np.ones(4)
    p1, m, v = S.adam(p, g, np.zeros(4), np.zeros(4), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_fits_a_linear_map():
    """Full-batch Adam on the network reduces the loss of a linear target by
    two orders of magnitude."""
    gen = workloads.SplitMix64(77)
    p = workloads.xavier_params(gen)
    g = np.random.default_rng(12)
    X = g.uniform(-1, 1, (128, 8))
    A = g.uniform(-0.5, 0.5, (8, 6))
    Y = X @ A
    m = v = np.zeros(S.N_PARAMS)
    L0 = S.loss_grad(p, X, Y)[0]
    for t in range(1, 601):
        L, gr = S.loss_grad(p, X, Y)
        p, m, v = S.adam(p, gr, m, v, t, 3e-3)
    assert S.loss_grad(p, X, Y)[0] < 1e-2 * L0


def test_xavier_bounds():
    p = S.unpack(workloads.xavier_params(workloads.SplitMix64(5)))
    for name, fi, fo in (("W1", 8, 64), ("W2", 64, 64), ("W3", 64, 6)):
        lim = math.sqrt(6 / (fi + fo))
        assert np.abs(p[name]).max() <= lim and np.abs(p[name]).max() > 0.9 * lim
        assert abs(p[name].mean()) < 0.1 * lim
    for b in ("b1", "b2", "b3"):
        assert not p[b].any()


def _rand_pose(g):
    q = g.standard_normal(4)
    return q / np.linalg.norm(q)


def test_features_are_frame_and_scale_invariant():
    g = np.random.default_rng(13)
    axes, q = (6.0, 2.0, 2.0), _rand_pose(g)
    F, T = g.standard_normal(3) * 1e-4, g.standard_normal(3) * 1e-3
    x, s = S.features(axes, q, F, T, (40, 40, 40))
    # rotate everything by Q: body-frame loads unchanged
    Qq = _rand_pose(g)
    Q = S.rotmat(Qq)
    q2 = np.array([Qq[0] * q[0] - Qq[1:] @ q[1:], *(Qq[0] * q[1:] + q[0] * Qq[1:] + np.cross(Qq[1:], q[1:]))])
    assert np.allclose(S.rotmat(q2), Q @ S.rotmat(q), atol=1e-14)
    x2, s2 = S.features(axes, q2, Q @ F, Q @ T, (40, 40, 40))
    assert np.allclose(x, x2, atol=1e-13) and abs(s - s2) < 1e-15
    # Stokes linearity: loads scaled by lambda keep x and scale s
    x3, s3 = S.features(axes, q, 7 * F, 7 * T, (40, 40, 40))
    assert np.allclose(x, x3, atol=1e-14) and abs(s3 - 7 * s) < 1e-14
    assert abs(np.linalg.norm(x[2:]) - 1) < 1e-14
    assert x[0] == pytest.approx(math.log(3)) and x[1] == pytest.approx(6 / 40)


def test_velocities_invert_targets():
    g = np.random.default_rng(14)
    axes, q = (5.0, 2.5, 2.0), _rand_pose(g)
    F, T = g.standard_normal(3) * 1e-4, g.standard_normal(3) * 1e-3
    U, W = g.standard_normal(3) * 1e-5, g.standard_normal(3) * 1e-6
    y = S.targets(U, W, axes, q, F, T, 1 / 6)
    U2, W2 = S.velocities(y, axes, q, F, T, 1 / 6)
    assert np.allclose(U2, U, rtol=1e-13, atol=0) and np.allclose(W2, W, rtol=1e-13, atol=0)


def test_sphere_targets_are_unit_mobility():
    """A sphere in an unbounded fluid moves with U = F / 6 pi mu R and
    Omega = T / 8 pi mu R^3: the normalised output equals the load inputs."""
    g = np.random.default_rng(15)
    axes, q = (3.0, 3.0, 3.0), _rand_pose(g)
    F, T = g.standard_normal(3) * 1e-4, g.standard_normal(3) * 1e-3
    U, W = S.unbounded_velocities(axes, q, F, T, 1 / 6)
    x, _ = S.features(axes, q, F, T, (40, 40, 40))
    assert np.allclose(S.targets(U, W, axes, q, F, T, 1 / 6), x[2:], atol=1e-13)


def test_resistance_functions_match_perrin():
    """Kim & Karrila's X^A, Y^A, X^C, Y^C against Perrin's friction
    coefficients of a prolate spheroid (Perrin 1934), a separately published
    form; and the sphere limit."""
    for r in (1.05, 1.5, 3.0, 5.0):
        a, b = r, 1.0
        c = math.sqrt(a * a - b * b)
        Sx = 2 / c * math.log((a + c) / b)
        fpar = 16 * math.pi * (a * a - b * b) / ((2 * a * a - b * b) * Sx - 2 * a)
        fperp = 32 * math.pi * (a * a - b * b) / ((2 * a * a - 3 * b * b) * Sx + 2 * a)
        rax = 32 * math.pi / 3 * (a * a - b * b) * b * b / (2 * a - b * b * Sx)
        rtr = 32 * math.pi / 3 * (a ** 4 - b ** 4) / ((2 * a * a - b * b) * Sx - 2 * a)
        XA, YA, XC, YC = S.kim_karrila(r)
        ref = (fpar / (6 * math.pi * a), fperp / (6 * math.pi * a), rax / (8 * math.pi * a ** 3),
               rtr / (8 * math.pi * a ** 3))
        assert np.allclose((XA, YA, XC, YC), ref, rtol=1e-9)
    assert np.allclose(S.kim_karrila(1 + 1e-5), 1.0, atol=1e-4)
    # the drift of the inclined r = 3 spheroid (Sec. III.B): 5.891 deg
    XA, YA, _, _ = S.kim_karrila(3.0)
    assert abs(45 - math.degrees(math.atan(XA / YA)) - 5.891) < 1e-3


def test_squirmer_speed_limits_and_series():
    """Eq. squirmervel pinned by what fixes it independently: the sphere's
    2 B1 / 3, the needle limit B1, the small-eccentricity series
    U_s / B1 = 2/3 + (2/15) e^2 + (2/35) e^4 + (2/63) e^6 + ... (from
    arcoth(1/e) = atanh(e) = e + e^3/3 + e^5/5 + ...), and the growth with the
    aspect ratio the paper's Fig. 8(a) shows; U_s is linear in B1."""
    assert S.squirmer_speed(1.0, 3e-3) == pytest.approx(2e-3, rel=1e-15)
    for e in (0.02, 0.05, 0.1):
        r = 1 / math.sqrt(1 - e * e)
        series = 2 / 3 + 2 / 15 * e ** 2 + 2 / 35 * e ** 4
        assert abs(S.squirmer_speed(r, 1.0) - series) < 0.04 * e ** 6 + 1e-14 / e ** 2
    assert abs(S.squirmer_speed(1e4, 1.0) - 1.0) < 1e-6
    speeds = [S.squirmer_speed(r, 1.0) for r in (1.0, 1.5, 2.0, 3.0, 5.0)]
    assert all(b > a for a, b in zip(speeds, speeds[1:]))
    assert S.squirmer_speed(2.0, -2e-3) == pytest.approx(-2 * S.squirmer_speed(2.0, 1e-3), rel=1e-15)


def test_squirmer_features_carry_the_propulsive_load():
    """A force-free squirmer enters the surrogate with the Stokes drag of its
    free swimming: for a sphere 6 pi mu R (2 B1 / 3) = 4 pi mu R B1 along its
    axis, so that a unit-mobility output is a sphere swimming at 2 B1 / 3;
    L is the box's volume per particle."""
    g = np.random.default_rng(21)
    q = _rand_pose(g)
    mu, R, B1 = 1 / 6, 3.0, 1e-3
    assert S.propulsive_force((R, R, R), B1, mu) == pytest.approx(4 * math.pi * mu * R * B1, rel=1e-14)
    x, s = S.features((R, R, R), q, np.zeros(3), np.zeros(3), (64, 64, 64), n_box=8, B1=B1, mu=mu)
    assert np.allclose(x[2:], [1, 0, 0, 0, 0, 0], atol=1e-15) and x[1] == pytest.approx(R / 32)
    U, W = S.velocities(np.array([1.0, 0, 0, 0, 0, 0]), (R, R, R), q, np.zeros(3), np.zeros(3), mu, B1=B1)
    assert np.allclose(U, S.rotmat(q)[:, 0] * 2 * B1 / 3, rtol=1e-13, atol=0) and not W.any()
    # prolate r = 2: the closed forms give the free swimming speed back
    axes = (5.0, 2.5, 2.5)
    U, _ = S.unbounded_velocities(axes, q, S.rotmat(q)[:, 0] * S.propulsive_force(axes, B1, mu), np.zeros(3), mu)
    assert np.allclose(U, S.rotmat(q)[:, 0] * S.squirmer_speed(2.0, B1), rtol=1e-13, atol=0)


def test_stokes_field_exact_properties():
    g = np.random.default_rng(16)
    U, W, R = g.standard_normal(3), g.standard_normal(3), 2.7
    # continuity with rigid motion on the sphere
    e = g.standard_normal((50, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    on = S.stokes_velocity(R * e * (1 + 1e-12), U, W, R)
    assert np.allclose(on, U + np.cross(W, R * e), atol=1e-9)
    # divergence free outside (central differences, h = 1e-4)
    d = e * g.uniform(1.2 * R, 5 * R, (50, 1))
    h = 1e-4
    div = sum((S.stokes_velocity(d + h * np.eye(3)[k], U, W, R)[:, k]
               - S.stokes_velocity(d - h * np.eye(3)[k], U, W, R)[:, k]) / (2 * h) for k in range(3))
    assert np.abs(div).max() < 1e-7
    # far field of pure translation: Stokeslet of force 6 pi mu R U, i.e. (3R/4r)(U + (U.e)e)
    far = 1e5 * e
    st = 0.75 * R / 1e5 * (U + (e @ U)[:, None] * e)
    assert np.allclose(S.stokes_velocity(far, U, 0 * W, R), st, rtol=1e-8, atol=0)
    # pure rotation: the rotlet, (R/r)^3 W x d at every distance outside
    assert np.allclose(S.stokes_velocity(d, 0 * U, W, R),
                       (R / np.linalg.norm(d, axis=1)[:, None]) ** 3 * np.cross(W, d), rtol=1e-13, atol=0)


def test_start_field_has_zero_total_momentum():
    shape = (20, 18, 22)
    owner = np.zeros(np.prod(shape), dtype=np.uint16)
    z, y, x = np.meshgrid(np.arange(22), np.arange(18), np.arange(20), indexing="ij")
    inside = ((x - 9.3) / 4) ** 2 + ((y - 8.6) / 2) ** 2 + ((z - 10.2) / 2) ** 2 < 1
    owner[inside.ravel()] = 1
    p = {"centre": (9.3, 8.6, 10.2), "axes": (4, 2, 2), "q": (1, 0, 0, 0), "F": (1e-4, -2e-5, 3e-5),
         "T": (0, 1e-4, 2e-4), "U": (1e-3, -2e-4, 5e-4), "W": (1e-5, 2e-5, -3e-5), "M": 4 / 3 * math.pi * 16}
    rho, u = S.start_state(shape, owner, [p], 1 / 6)
    fl = owner == 0
    tot = (rho[fl, None] * u[fl]).sum(0) + p["M"] * np.array(p["U"])
    assert np.abs(tot).max() < 1e-15 * np.prod(shape)
    assert abs(rho[fl].sum() - fl.sum()) < 1e-12 and np.all(rho[~fl] == 1.0)
    assert np.abs(rho - 1).max() > 1e-6   # the pressure is there
    # solid nodes move rigidly
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)[owner == 1]
    rig = np.array(p["U"]) + np.cross(p["W"], pos - np.array(p["centre"]))
    assert np.allclose(u[owner == 1], rig, atol=1e-18)
    f = S.equilibrium(1.0, u)
    assert np.allclose(f.sum(1), 1.0, atol=1e-15)


def _ball(N):
    n = np.arange(-N, N + 1)
    X, Y, Z = np.meshgrid(n, n, n, indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(float)
    r = np.linalg.norm(v, axis=1)
    return v[(r > 0) & (r <= N)]


def test_periodic_modes_reproduce_hasimoto():
    """Summed over all wave vectors (a ball |n| <= 48 plus the isotropic
    continuum estimate of the rest, 1 / (6 pi^2 mu R^2 k_max) per unit force)
    and averaged over the sphere (one more sinc(kR)), the periodic modes give
    the velocity of a simple-cubic array of spheres under a force, which
    Hasimoto's expansion fixes: U / U_Stokes = 1 - 2.837297 x + 4.19 x^3,
    x = R/L.  The sphere model (uniform traction) may differ at O(x^3)."""
    n = _ball(48)
    k = 2 * np.pi * n
    kk = np.sqrt((k * k).sum(1))
    for x in (0.03, 0.05, 0.1, 0.15):
        u = S.periodic_modes(k, (1.0, 0, 0), (0, 0, 0), x, 1.0, 1.0)
        U = (u[:, 0].real * np.sin(kk * x) / (kk * x)).sum() + 1 / (6 * math.pi ** 2 * x * x * 2 * math.pi * 48)
        ratio = U * 6 * math.pi * x
        assert abs(ratio - (1 - 2.837297 * x + 4.19 * x ** 3)) < 2e-3, (x, ratio)


def test_periodic_modes_rotlet_near_field():
    """Near a small sphere turned by a torque, the summed periodic modes give
    the free-space rotlet T x d / (8 pi mu r^3) up to the images' O(1/V)
    correction."""
    n = _ball(48)
    k = 2 * np.pi * n
    R, T = 0.05, np.array([0.0, 0.0, 1.0])
    u = S.periodic_modes(k, (0, 0, 0), T, R, 1.0, 1.0)
    for d in (np.array([0.12, 0.03, 0.0]), np.array([0.1, -0.05, 0.04])):
        v = (u * np.exp(1j * (k @ d))[:, None]).sum(0).real
        ref = np.cross(T, d) / (8 * math.pi * np.linalg.norm(d) ** 3)
        assert np.abs(v - ref).max() < 0.25 * np.linalg.norm(np.cross(T, d)) + 0.01 * np.linalg.norm(ref)


def test_start_field_low_modes_are_periodic():
    """The start velocity's and pressure's modes |n_i| <= 2 equal the
    periodic solution's and the rest equal the free field's (before the
    momentum shift, on a box with no particle nodes; the pressure read back
    from the density as (rho - 1) / 3)."""
    shape, mu = (20, 18, 22), 1 / 6
    q = np.array([0.9, 0.2, -0.3, 0.25]) / np.linalg.norm([0.9, 0.2, -0.3, 0.25])
    part = {"centre": (9.3, 8.6, 10.2), "axes": (4, 2, 2), "q": q, "F": (1e-4, -2e-5, 3e-5),
            "T": (0, 1e-4, 2e-4), "U": (0, 0, 0), "W": (0, 0, 0), "M": 0.0}
    owner = np.zeros(np.prod(shape), dtype=np.uint16)
    rho, u = S.start_state(shape, owner, [part], mu)
    _, uf, pf = S.free_field(shape, [part], mu, pressure=True)
    N = np.prod(shape)
    args = (shape, part["centre"], part["F"], part["T"], S.req(part["axes"]), mu, part["axes"], part["q"])
    # the pressure read back from rho ~ 1 carries its rounding, ~1e-16 absolute
    for field, free, pressure, floor in ((u, uf, False, 0.0), ((rho - 1) / 3, pf, True, 1e-16)):
        A = np.fft.fftn(field.reshape(22, 18, 20, -1), axes=(0, 1, 2)) / N
        B = np.fft.fftn(free.reshape(22, 18, 20, -1), axes=(0, 1, 2)) / N
        ns, c = S.periodic_coefficients(*args, pressure=pressure)
        c = c.reshape(len(ns), -1)
        for n, cn in zip(ns, c):
            assert np.allclose(A[n[2] % 22, n[1] % 18, n[0] % 20], cn, rtol=0,
                               atol=1e-12 * np.abs(c).max() + floor)
        mask = np.ones((22, 18, 20), bool)
        for n in ns + [(0, 0, 0)]:
            mask[n[2] % 22, n[1] % 18, n[0] % 20] = False
        assert np.allclose(A[mask], B[mask], rtol=0, atol=1e-12 * np.abs(B).max() + floor)
    # the mean momentum (M = 0 here) and the mean density change are zero
    assert np.abs((rho[:, None] * u).mean(0)).max() < 1e-15
    assert abs((rho - 1).mean()) < 1e-16


def _spheroid_case(g, axes):
    q = g.standard_normal(4)
    q /= np.linalg.norm(q)
    return q, g.standard_normal(3), g.standard_normal(3) * axes[0]


SPHEROIDS = [(6.0, 3.0, 3.0), (10.0, 2.0, 2.0), (20.0, 4.0, 4.0), (4.2, 4.0, 4.0), (3.003, 3.0, 3.0)]


@pytest.mark.parametrize("axes", SPHEROIDS)
def test_spheroid_flow_meets_the_body(axes):
    """On the surface the line-singularity flow equals the rigid motion with
    the resistance functions' velocities (Kim & Karrila's X^A, Y^A, X^C, Y^C,
    pinned to Perrin's formulas above): together with decay at infinity and
    each singularity solving the Stokes equations, this fixes the flow as the
    unique creeping flow of the body moving under (F, T).  A wrong strength,
    sign or term breaks it."""
    g = np.random.default_rng(40)
    q, F, T = _spheroid_case(g, axes)
    mu = 1 / 6
    a, b, _ = axes
    th, ph = g.uniform(0, math.pi, 300), g.uniform(0, 2 * math.pi, 300)
    d = np.stack([a * np.cos(th), b * np.sin(th) * np.cos(ph), b * np.sin(th) * np.sin(ph)], 1) @ S.rotmat(q).T
    U, W = S.unbounded_velocities(axes, q, F, T, mu)
    for load in ((F, 0 * T), (0 * F, T)):
        Ul, Wl = S.unbounded_velocities(axes, q, *load, mu)
        u = S.spheroid_flow(d * (1 + 1e-12), axes, q, *load, mu)
        rig = Ul + np.cross(Wl, d)
        assert np.abs(u - rig).max() < 1e-10 * np.abs(rig).max()


@pytest.mark.parametrize("axes", SPHEROIDS[:3])
def test_spheroid_flow_is_solenoidal_and_decays_as_the_load(axes):
    """Divergence free outside the body (central differences); far away the
    flow of a force is its Stokeslet F / (8 pi mu) (I / r + d d / r^3), and
    that of a torque about the axis its rotlet T x d / (8 pi mu r^3)."""
    g = np.random.default_rng(41)
    q, F, T = _spheroid_case(g, axes)
    mu = 1 / 6
    a = axes[0]
    e = g.standard_normal((40, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    d = e * g.uniform(1.3 * a, 3 * a, (40, 1))
    h = 1e-4
    div = sum((S.spheroid_flow(d + h * np.eye(3)[k], axes, q, F, T, mu)[:, k]
               - S.spheroid_flow(d - h * np.eye(3)[k], axes, q, F, T, mu)[:, k]) / (2 * h) for k in range(3))
    scale = np.abs(S.spheroid_flow(d, axes, q, F, T, mu)).max() / a
    assert np.abs(div).max() < 1e-7 * scale
    far = 1e4 * a * e
    r = np.linalg.norm(far, axis=1)[:, None]
    st = (F / r + (far @ F)[:, None] * far / r ** 3) / (8 * math.pi * mu)
    assert np.allclose(S.spheroid_flow(far, axes, q, F, 0 * T, mu), st, rtol=0, atol=1e-7 * np.abs(st).max())
    p = S.rotmat(q)[:, 0]
    Ta = (T @ p) * p
    rot = np.cross(Ta, far) / (8 * math.pi * mu * r ** 3)
    assert np.allclose(S.spheroid_flow(far, axes, q, 0 * F, Ta, mu), rot, rtol=0, atol=1e-7 * np.abs(rot).max())


def test_spheroid_flow_tends_to_the_sphere():
    """Just above E_LINE the spheroid's flow is the sphere's Stokes solution
    and rotlet to O(e^2)."""
    g = np.random.default_rng(42)
    a = 3.0
    axes = (a, a * math.sqrt(1 - (2 * S.E_LINE) ** 2), a * math.sqrt(1 - (2 * S.E_LINE) ** 2))
    q, F, T = _spheroid_case(g, axes)
    mu = 0.1
    e = g.standard_normal((40, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    d = e * g.uniform(1.05 * a, 4 * a, (40, 1))
    u = S.spheroid_flow(d, axes, q, F, T, mu)
    ref = S.stokes_velocity(d, F / (6 * math.pi * mu * a), T / (8 * math.pi * mu * a ** 3), a)
    assert np.abs(u - ref).max() < 1e-6 * np.abs(ref).max()


def test_translating_spheroid_is_a_single_layer_of_the_mapped_sphere():
    """Outside a translating prolate spheroid the flow equals the Stokeslets
    of its force spread over the surface as the uniform measure on the unit
    sphere mapped by diag(a, b, b) in the body frame (the reading behind the
    periodic coefficients' form factor sinc(|diag(a, b, c) R^T k|), which is
    that measure's Fourier transform).  Quadrature over the unit sphere:
    Gauss-Legendre in cos(theta), trapezoid in phi."""
    g = np.random.default_rng(43)
    axes = (7.0, 2.5, 2.5)
    q, F, _ = _spheroid_case(g, axes)
    mu = 0.2
    Rm = S.rotmat(q)
    ct, wt = np.polynomial.legendre.leggauss(160)
    ph = np.arange(320) * 2 * math.pi / 320
    st = np.sqrt(1 - ct * ct)
    n = np.stack([np.outer(ct, np.ones_like(ph)), np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph))], -1).reshape(-1, 3)
    w = (np.outer(wt, np.ones_like(ph)) * (2 * math.pi / 320)).ravel() / (4 * math.pi)
    y = (n * np.asarray(axes)) @ Rm.T
    assert abs(w.sum() - 1) < 1e-13
    pts = np.array([[0.0, 0.0, 4.0], [9.0, 1.0, -2.0], [-3.0, 5.0, 2.0], [2.0, -2.0, -6.0]])
    u = S.spheroid_flow(pts, axes, q, F, 0 * F, mu)
    for x, ux in zip(pts, u):
        r = x - y
        R = np.linalg.norm(r, axis=1)[:, None]
        G = F / R + (r @ F)[:, None] * r / R ** 3
        v = (w[:, None] * G).sum(0) / (8 * math.pi * mu)
        assert np.abs(v - ux).max() < 1e-9 * np.abs(ux).max()
    # the measure's transform is sinc(|diag(a, b, b) R^T k|)
    for k in (np.array([0.3, -0.2, 0.5]), np.array([0.05, 0.4, 0.1])):
        ft = (w * np.exp(-1j * (y @ k))).sum()
        ka = np.linalg.norm((k @ Rm) * np.asarray(axes))
        assert abs(ft - math.sin(ka) / ka) < 1e-12


@pytest.mark.parametrize("axes", [(6.0, 3.0, 3.0), (10.0, 2.0, 2.0), (3.0, 3.0, 3.0)])
def test_start_pressure_balances_the_viscous_stress(axes):
    """Outside the body the free flow's pressure and velocity satisfy the
    Stokes equations, grad p = mu lap u (second-order central differences,
    h = 3e-3; the truncation error is ~h^2 of the fourth derivatives), for a
    spheroid under force and torque and for the sphere; far away a force's
    pressure is F.d / (4 pi r^3) (a torque's stresslet adds O(1/r^3))."""
    g = np.random.default_rng(44)
    q, F, T = _spheroid_case(g, axes)
    part = {"axes": axes, "q": q, "F": F, "T": T}
    mu = 0.3
    a = axes[0]
    e = g.standard_normal((30, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    d = e * g.uniform(1.4 * a, 2.5 * a, (30, 1))
    h = 3e-3
    I = np.eye(3)
    grad = np.stack([(S.particle_pressure(d + h * I[k], part, mu) - S.particle_pressure(d - h * I[k], part, mu))
                     / (2 * h) for k in range(3)], 1)
    lap = sum(S.particle_flow(d + h * I[k], part, mu) + S.particle_flow(d - h * I[k], part, mu)
              for k in range(3)) - 6 * S.particle_flow(d, part, mu)
    lap /= h * h
    assert np.abs(grad - mu * lap).max() < 1e-5 * np.abs(grad).max()
    far = 1e4 * a * e
    ref = (far @ F) / (4 * math.pi * np.linalg.norm(far, axis=1) ** 3)
    force_only = dict(part, T=np.zeros(3))
    assert np.allclose(S.particle_pressure(far, force_only, mu), ref, rtol=0, atol=1e-6 * np.abs(ref).max())


def test_periodic_pressure_modes_near_a_small_sphere():
    """Summed over all wave vectors, the periodic pressure of a force spread
    on a small sphere gives the point force's F.d / (4 pi r^3) near it, up to
    the images' O(1/V) correction (the mean force is balanced by the
    box-wide counter-force, which drives no pressure)."""
    n = _ball(48)
    k = 2 * np.pi * n
    F = np.array([0.3, -1.0, 0.5])
    pk = S.periodic_pressure_modes(k, F, 0.05, 1.0)
    for d in (np.array([0.12, 0.03, 0.0]), np.array([0.1, -0.05, 0.04])):
        v = (pk * np.exp(1j * (k @ d))).sum().real
        ref = (F @ d) / (4 * math.pi * np.linalg.norm(d) ** 3)
        assert abs(v - ref) < 0.02 * abs(ref) + 0.05


@pytest.mark.parametrize("axes", [(7.0, 2.5, 2.5), (5.0, 4.0, 4.0)])
def test_rotating_spheroid_is_a_linear_single_layer(axes):
    """Outside a prolate spheroid turned by a torque the flow equals the
    Stokeslets of the traction sigma C x, sigma the unit sphere's uniform
    measure mapped by diag(a, b, b), C = 3 Q^T A^-2 with Q the first moment
    that rotation_traction carries (the torque's antisymmetric part and the
    line solution's stresslet); that traction has the torque T, and its
    transform is rotation_traction's -3 i (Q^T k) j1(kappa) / kappa.
    Quadrature over the unit sphere: Gauss-Legendre in cos(theta),
    trapezoid in phi."""
    g = np.random.default_rng(45)
    q = g.standard_normal(4)
    q /= np.linalg.norm(q)
    T = g.standard_normal(3)
    mu = 0.2
    Rm = S.rotmat(q)
    QT = np.stack([S.rotation_traction(np.eye(3)[j][None], T, 1.0, axes, q)[0][0] for j in range(3)], 1)
    A2 = Rm @ np.diag(np.asarray(axes) ** 2) @ Rm.T
    C = 3 * QT @ np.linalg.inv(A2)
    ct, wt = np.polynomial.legendre.leggauss(160)
    ph = np.arange(320) * 2 * math.pi / 320
    st = np.sqrt(1 - ct * ct)
    n = np.stack([np.outer(ct, np.ones_like(ph)), np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph))], -1).reshape(-1, 3)
    w = (np.outer(wt, np.ones_like(ph)) * (2 * math.pi / 320)).ravel() / (4 * math.pi)
    y = (n * np.asarray(axes)) @ Rm.T
    f = y @ C.T
    assert np.abs((w[:, None] * np.cross(y, f)).sum(0) - T).max() < 1e-12 * np.abs(T).max()
    a = axes[0]
    pts = np.array([[0.0, 0.0, 1.5 * a], [1.6 * a, 1.0, -2.0], [-3.0, 1.5 * a, 2.0]])
    u = S.spheroid_flow(pts, axes, q, np.zeros(3), T, mu)
    for x, ux in zip(pts, u):
        r = x - y
        R = np.linalg.norm(r, axis=1)[:, None]
        G = f / R + (r * f).sum(1)[:, None] * r / R ** 3
        v = (w[:, None] * G).sum(0) / (8 * math.pi * mu)
        assert np.abs(v - ux).max() < 1e-9 * np.abs(ux).max()
    for k in (np.array([0.3, -0.2, 0.5]), np.array([0.05, 0.4, 0.1])):
        ft = (w[:, None] * f * np.exp(-1j * (y @ k))[:, None]).sum(0)
        gk, j1k = S.rotation_traction(k[None], T, 1.0, axes, q)
        assert np.abs(ft - (-3j * gk[0] * j1k[0])).max() < 1e-12 * np.abs(ft).max()
