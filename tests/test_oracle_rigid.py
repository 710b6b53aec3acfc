"""Pins of the oracle's rigid-body pieces (Sec. II.C, II.D, III.D): lab-frame
inertia (eq. Irot) against R diag(I) R^T from scipy, its time derivative
(eq. Irotdiff) against the commutator closed form and a central difference,
the exponential quaternion update (eqs. qnplus0/1), the 6x6 elimination, and
the squirmer slip (eq. squirmer) against the textbook spherical squirmer."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def rot(q):
    q = np.asarray(q, float)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def rand_q(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def test_inertia_identity_and_quarter_turn(orc):
    Ib = np.array([1.0, 2.0, 3.5])
    assert np.allclose(orc.inertia_lab([1, 0, 0, 0], Ib), np.diag(Ib), atol=1e-15)
    qz = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]
    assert np.allclose(orc.inertia_lab(qz, Ib), np.diag([2.0, 1.0, 3.5]), atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_inertia_lab_is_rotated_tensor(orc, seed):
    rng = np.random.default_rng(seed)
    q = rand_q(rng)
    Ib = rng.random(3) + 0.5
    R = rot(q)
    I = orc.inertia_lab(q, Ib)
    assert np.allclose(I, R @ np.diag(Ib) @ R.T, rtol=0, atol=1e-14)
    assert np.isclose(np.trace(I), Ib.sum(), rtol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_inertia_rate(orc, seed):
    """dI/dt from the four product-rule terms equals [W]x I' - I' [W]x, and a
    central difference of I'(q(t)) along q(t) = exp(W t / 2) q."""
    rng = np.random.default_rng(10 + seed)
    q = rand_q(rng)
    Ib = rng.random(3) + 0.5
    W = rng.standard_normal(3) * 0.3
    Id = orc.inertia_dot(q, Ib, W)
    I = orc.inertia_lab(q, Ib)
    assert np.allclose(Id, skew(W) @ I - I @ skew(W), rtol=0, atol=1e-14)
    h = 1e-5
    R0 = Rotation.from_quat([q[1], q[2], q[3], q[0]])
    Ip = (Rotation.from_rotvec(W * h) * R0).as_matrix()
    Im = (Rotation.from_rotvec(-W * h) * R0).as_matrix()
    fd = (Ip @ np.diag(Ib) @ Ip.T - Im @ np.diag(Ib) @ Im.T) / (2 * h)
    assert np.allclose(Id, fd, rtol=0, atol=1e-8)


def test_quaternion_constant_spin(orc):
    """Constant Omega = (0,0,w): q_n = (cos(n w/2), 0, 0, sin(n w/2))."""
    w = 0.0123
    q = np.array([1.0, 0, 0, 0])
    for n in range(1, 2001):
        q = orc.quat_update(q, [0, 0, w])
    assert np.allclose(q, [np.cos(2000 * w / 2), 0, 0, np.sin(2000 * w / 2)], atol=1e-12)


def test_quaternion_norm_without_renormalisation(orc):
    """The exponential update keeps |q| = 1 (end of Sec. II.C) over 10^5 steps."""
    rng = np.random.default_rng(5)
    q = rand_q(rng)
    Ws = rng.standard_normal((100000, 3)) * 0.05
    for W in Ws:
        q = orc.quat_update(q, W)
    assert abs(np.linalg.norm(q) - 1) < 1e-12


def test_quaternion_update_matches_rotation_composition(orc):
    rng = np.random.default_rng(8)
    q = rand_q(rng)
    W = rng.standard_normal(3) * 0.2
    qn = orc.quat_update(q, W)
    R = (Rotation.from_rotvec(W) * Rotation.from_quat([q[1], q[2], q[3], q[0]])).as_matrix()
    assert np.allclose(rot(qn), R, atol=1e-14)
    assert np.allclose(orc.quat_update(q, [0, 0, 0]), q, atol=0)


def test_solve6(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        A = rng.standard_normal((6, 6)) + 4 * np.eye(6)
        b = rng.standard_normal(6)
        x = orc.solve6(A, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-13)
    # needs pivoting: zero leading entry
    A = rng.standard_normal((6, 6))
    A[0, 0] = 0.0
    b = rng.standard_normal(6)
    assert np.allclose(orc.solve6(A, b), np.linalg.solve(A, b), rtol=1e-10)
    with pytest.raises(ZeroDivisionError):
        orc.solve6(np.zeros((6, 6)), b)


def test_squirmer_sphere_limit(orc):
    """a = b = c: slip is B1 sin(th)(1 + beta cos(th)) e_theta (Blake squirmer),
    with th measured from the body x axis e and e_theta pointing away from e."""
    R = 3.0
    B1, B2 = 1e-3, -2e-3
    q = np.array([0.8, 0.1, -0.3, 0.5])
    q /= np.linalg.norm(q)
    e = rot(q)[:, 0]
    rng = np.random.default_rng(4)
    for _ in range(20):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        d = R * n
        us = orc.squirmer_slip([R, R, R], q, B1, B2, d)
        ct = n @ e
        st = np.sqrt(1 - ct * ct)
        eth = (ct * n - e) / st
        assert np.allclose(us, B1 * st * (1 + (B2 / B1) * ct) * eth, atol=1e-15)


def test_squirmer_slip_is_tangential(orc):
    """On the spheroid surface the slip has no normal component (eq. squirmer)."""
    a, b = 5.0, 2.5
    q = np.array([0.6, -0.2, 0.7, 0.3])
    q /= np.linalg.norm(q)
    R = rot(q)
    rng = np.random.default_rng(6)
    for _ in range(20):
        v = rng.standard_normal(3)
        v /= np.sqrt((v[0] / a) ** 2 + (v[1] / b) ** 2 + (v[2] / b) ** 2)   # body surface point
        nrm = np.array([v[0] / a ** 2, v[1] / b ** 2, v[2] / b ** 2])
        us = orc.squirmer_slip([a, b, b], q, 1e-3, 5e-4, R @ v)
        assert abs((R @ nrm) @ us) < 1e-15
        assert np.linalg.norm(us) > 0


def test_squirmer_spheroidal_coordinate_on_the_surface(orc):
    """Eq. squirmer on a prolate spheroid (a, b, b), eps > 0, B1 = 0: the slip
    is -B2 zeta (s . e) s with zeta = z / a on the surface (the foci sit at
    +-a eps on the axis, and on the ellipse the focal distances differ by
    2 eps z) and s the unit meridian tangent, built here from the ellipse
    parametrisation (z, rho) = (a cos t, b sin t), d/dt = (-a sin t, b cos t).
    A wrong focal factor in zeta changes the B2 mode by tens of percent."""
    rng = np.random.default_rng(11)
    for a, b in ((5.0, 2.5), (6.0, 2.0), (3.0, 2.9)):
        q = rand_q(rng)
        R = rot(q)
        for _ in range(25):
            t = rng.uniform(0.05, np.pi - 0.05)
            phi = rng.uniform(0, 2 * np.pi)
            z, rho = a * np.cos(t), b * np.sin(t)
            perp = np.array([0.0, np.cos(phi), np.sin(phi)])  # body frame, e = body x
            x_body = np.array([z, 0, 0]) + rho * perp
            s = np.array([-a * np.sin(t), 0, 0]) + b * np.cos(t) * perp
            s /= np.linalg.norm(s)
            for B1, B2 in ((0.0, 1e-3), (7e-4, -2e-3)):
                expect = R @ (-(B1 + B2 * z / a) * s[0] * s)
                got = orc.squirmer_slip([a, b, b], q, B1, B2, R @ x_body)
                assert np.allclose(got, expect, rtol=1e-12, atol=1e-17), (a, b, t, B1, B2)


def test_squirmer_spheroidal_coordinate_off_the_surface(orc):
    """Off the surface zeta is the angular prolate spheroidal coordinate of
    the point, cos(v) in z = f cosh(u) cos(v), rho = f sinh(u) sin(v) with
    f = a eps: with l = cosh^2 u and h = cos^2 v, l h = (z/f)^2 and
    l + h = 1 + (z/f)^2 + (rho/f)^2, so h is the smaller root of a quadratic
    (an algebraic route, not the focal-distance formula of the paper); s is
    the surface tangent at the point's axial coordinate (clamped to [-a, a],
    reading R11)."""
    rng = np.random.default_rng(12)
    a, b = 5.0, 2.5
    f = a * np.sqrt(1 - (b / a) ** 2)
    for _ in range(40):
        z, rho = rng.uniform(-a, a), rng.uniform(0.3, 2 * b)
        Z2, R2 = (z / f) ** 2, (rho / f) ** 2
        ssum = 1 + Z2 + R2
        h = (ssum - np.sqrt(ssum * ssum - 4 * Z2)) / 2
        zeta = np.sign(z) * np.sqrt(h)
        ct = z / a
        s = np.array([-a * np.sqrt(1 - ct * ct), b * ct, 0.0])
        s /= np.linalg.norm(s)
        got = orc.squirmer_slip([a, b, b], [1, 0, 0, 0], 0.0, 1e-3, [z, rho, 0.0])
        assert np.allclose(got, -1e-3 * zeta * s[0] * s, rtol=1e-11, atol=1e-18), (z, rho)
