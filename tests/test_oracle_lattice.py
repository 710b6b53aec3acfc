"""Pins of the oracle's lattice Boltzmann fluid (Sec. II.A) against facts that
do not come from the oracle: lattice isotropy, exact moment identities, the
viscosity relation nu = (tau - 1/2)/3, the streaming permutation and the
Couette flow between moving walls (an exact steady solution)."""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def feq_field(c, w, rho, u):
    cu = u @ c.T
    uu = (u * u).sum(1)[:, None]
    return rho * w[None, :] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def test_d3q19_isotropy(orc):
    """Textbook D3Q19 (Sec. II.A): sum w = 1, odd moments vanish, second moment
    c_s^2 I with c_s^2 = 1/3, fourth moment c_s^4 (dd + dd + dd)."""
    c, w = orc.lattice()
    assert np.isclose(w.sum(), 1.0, rtol=0, atol=1e-15)
    assert np.abs(w @ c).max() < 1e-16
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, np.eye(3) / 3, atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    m3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(m3).max() < 1e-16
    # header order: opposite of odd i is i+1, rest vector first
    assert (c[0] == 0).all()
    for i in range(1, 19, 2):
        assert (c[i] == -c[i + 1]).all()


def test_equilibrium_moments(orc):
    """f_eq reproduces rho, rho u and rho c_s^2 I + rho u u exactly (Sec. II.A)."""
    c, _ = orc.lattice()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        f = orc.equilibrium(rho, u)
        assert np.isclose(f.sum(), rho, rtol=1e-14)
        assert np.allclose(f @ c, rho * u, rtol=0, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.allclose(P, rho * np.eye(3) / 3 + rho * np.outer(u, u), rtol=0, atol=1e-15)


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("bgk", 1.0), ("trt", 0.7), ("trt", 1.3),
                                      ("reg", 0.9), ("reg", 1.0)])
def test_collision_invariants(orc, coll, tau):
    """Collision conserves mass and momentum; BGK scales f - f_eq by 1 - 1/tau
    (reading of the garbled sign in Sec. II.A); the ghost-mode scheme keeps
    only hydrodynamic modes with the stress deviation scaled by 1 - 1/tau."""
    c, w = orc.lattice()
    s = orc.OracleSim((4, 4, 4), coll, tau)
    rng = np.random.default_rng(7)
    for _ in range(10):
        rho = 1 + 0.01 * rng.standard_normal()
        u = 0.02 * rng.standard_normal(3)
        f = orc.equilibrium(rho, u) + 1e-3 * w * rng.standard_normal(19)
        out = s.collide_node(f)
        rho_in, j_in = f.sum(), f @ c
        assert np.isclose(out.sum(), rho_in, rtol=1e-14)
        assert np.allclose(out @ c, j_in, rtol=0, atol=1e-15)
        feq = orc.equilibrium(rho_in, j_in / rho_in)
        if coll == "bgk":
            assert np.allclose(out - feq, (1 - 1 / tau) * (f - feq), rtol=0, atol=1e-15)
        if coll == "reg":
            # stress: Pi* - Pi_eq = (1 - 1/tau)(Pi - Pi_eq)
            P = lambda g: np.einsum("i,ia,ib->ab", g, c, c)
            assert np.allclose(P(out) - P(feq), (1 - 1 / tau) * (P(f) - P(feq)), atol=1e-15)
            # ghost content is zero: out lies in span{w, w c, w c c}
            basis = [w] + [w * c[:, a] for a in range(3)] + \
                    [w * c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)]
            B = np.array(basis).T
            coef, *_ = np.linalg.lstsq(B, out, rcond=None)
            assert np.abs(B @ coef - out).max() < 1e-15
        if tau == 1.0:
            assert np.allclose(out, feq, rtol=0, atol=1e-15)


def test_trt_reduces_to_bgk(orc):
    """TRT with tau- = tau+ (Lambda = (tau-1/2)^2) is BGK."""
    tau = 0.85
    s1 = orc.OracleSim((4, 4, 4), "bgk", tau)
    s2 = orc.OracleSim((4, 4, 4), "trt", tau, magic=(tau - 0.5) ** 2)
    rng = np.random.default_rng(3)
    _, w = orc.lattice()
    f = orc.equilibrium(1.0, [0.01, -0.02, 0.005]) + 1e-3 * w * rng.standard_normal(19)
    assert np.allclose(s1.collide_node(f), s2.collide_node(f), rtol=0, atol=1e-16)


def test_streaming_is_a_periodic_shift(orc):
    """Streaming moves f_i by c_i with periodic wrap: np.roll of each population."""
    c, _ = orc.lattice()
    nx, ny, nz = 7, 5, 6
    s = orc.OracleSim((nx, ny, nz))
    rng = np.random.default_rng(0)
    f = rng.random((nx * ny * nz, 19))
    s.set_f(f)
    s.stream_only()
    g = s.get_f()
    for i in range(19):
        a = f[:, i].reshape(nz, ny, nx)
        rolled = np.roll(a, shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(rolled.reshape(-1), g[:, i])


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("trt", 0.8), ("reg", 0.8), ("bgk", 1.3),
                                      ("trt", 1.3)])
def test_shear_wave_viscosity(orc, coll, tau):
    """A shear wave decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3 (Sec. II.A).
    Tolerance 1%: lattice dispersion at k = 2 pi/64 is far below it, while any
    slip in the tau -> nu relation is tens of percent."""
    c, w = orc.lattice()
    L = 64
    s = orc.OracleSim((2, L, 2), coll, tau)
    y = (np.arange(s.n) // 2) % L
    u = np.zeros((s.n, 3))
    u[:, 0] = 1e-4 * np.sin(2 * np.pi * y / L)
    s.set_f(feq_field(c, w, 1.0, u))
    amps = []
    for n in (100, 400):
        s.step(n)
        _, uu = s.fields()
        amps.append((uu[:, 0] * np.sin(2 * np.pi * y / L)).sum() * 2 / s.n)
    k2 = (2 * np.pi / L) ** 2
    nu = np.log(amps[0] / amps[1]) / (400 * k2)
    assert abs(nu / ((tau - 0.5) / 3) - 1) < 0.01


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("trt", 0.8), ("reg", 1.2)])
def test_couette_between_moving_walls(orc, coll, tau):
    """Walls at y=0 and y=ny-1 moving at -U and +U (Sec. III.C set-up): the
    linear profile between the half-way planes is an exact steady solution of
    link bounce-back with the moving-boundary term of eq. fb."""
    ny, U = 12, 0.01
    s = orc.OracleSim((4, ny, 4), coll, tau, walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0),
                      init="couette")
    m0 = s.mass()
    s.step(300)
    rho, u = s.fields()
    y = (np.arange(s.n) // 4) % ny
    fl = (y > 0) & (y < ny - 1)
    ex = -U + 2 * U * (y - 0.5) / (ny - 2)
    assert np.abs(u[fl, 0] - ex[fl]).max() < 1e-12 * U * 100
    assert np.abs(u[fl, 1:]).max() < 1e-14
    assert abs(s.mass() / m0 - 1) < 1e-12


def test_couette_develops_from_rest(orc):
    """Started from rest, the wall-driven flow converges to the same line."""
    ny, U = 10, 0.01
    s = orc.OracleSim((2, ny, 2), "trt", 1.0, walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0))
    s.step(3000)
    _, u = s.fields()
    y = (np.arange(s.n) // 2) % ny
    fl = (y > 0) & (y < ny - 1)
    ex = -U + 2 * U * (y - 0.5) / (ny - 2)
    assert np.abs(u[fl, 0] - ex[fl]).max() < 1e-6 * U
