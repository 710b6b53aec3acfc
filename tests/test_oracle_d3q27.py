"""Pins of the oracle's D3Q27 lattice (the paper's lattice-independence check,
Sec. III.A, Fig. 3d) against facts that do not come from the oracle: the
velocity set is the full 3 x 3 x 3 stencil, the weights are the tensor
product of the one-dimensional weights (2/3, 1/6, 1/6), the lattice is
isotropic to the orders the D3Q19 tests check plus a sixth-order moment
D3Q19 lacks, equilibrium moments, collision invariants, streaming as
np.roll, the viscosity relation, the exact Couette solution, conservation
with a moving particle, Hasimoto's sphere drag, and D3Q19 agreeing with
D3Q27 on a settling spheroid."""
import itertools

import numpy as np
import pytest
from scipy.optimize import brentq

from test_oracle_lattice import feq_field
from test_oracle_physics import hasimoto, total_momentum

pytestmark = pytest.mark.filterwarnings("ignore")


def test_d3q27_velocity_set_and_weights(orc):
    c, w = orc.lattice(27)
    assert sorted(map(tuple, c)) == sorted(itertools.product((-1, 0, 1), repeat=3))
    c19, w19 = orc.lattice(19)
    assert np.array_equal(c[:19], c19)          # D3Q19 order first, corners appended
    assert (c[0] == 0).all()
    for i in range(1, 27, 2):
        assert (c[i] == -c[i + 1]).all()         # opposite of odd i is i + 1
    w1 = {0: 2 / 3, 1: 1 / 6, -1: 1 / 6}
    for ci, wi in zip(c, w):
        assert np.isclose(wi, w1[ci[0]] * w1[ci[1]] * w1[ci[2]], rtol=1e-15, atol=0)


def test_d3q27_isotropy(orc):
    c, w = orc.lattice(27)
    assert np.isclose(w.sum(), 1.0, rtol=0, atol=1e-15)
    assert np.abs(w @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-15)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-15)
    # sixth order: sum w cx^2 cy^2 cz^2 = c_s^6 = 1/27 (zero on D3Q19, no corners)
    m6 = (w * c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2).sum()
    assert np.isclose(m6, 1 / 27, rtol=1e-14)
    c19, w19 = orc.lattice(19)
    assert (w19 * c19[:, 0] ** 2 * c19[:, 1] ** 2 * c19[:, 2] ** 2).sum() == 0


def test_d3q27_equilibrium_moments(orc):
    c, _ = orc.lattice(27)
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        f = orc.equilibrium(rho, u, 27)
        assert np.isclose(f.sum(), rho, rtol=1e-14)
        assert np.allclose(f @ c, rho * u, rtol=0, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.allclose(P, rho * np.eye(3) / 3 + rho * np.outer(u, u), rtol=0, atol=1e-15)


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("bgk", 1.0), ("trt", 0.7), ("reg", 0.9), ("reg", 1.0)])
def test_d3q27_collision_invariants(orc, coll, tau):
    c, w = orc.lattice(27)
    s = orc.OracleSim((4, 4, 4), coll, tau, lattice=27)
    rng = np.random.default_rng(5)
    for _ in range(10):
        rho = 1 + 0.01 * rng.standard_normal()
        u = 0.02 * rng.standard_normal(3)
        f = orc.equilibrium(rho, u, 27) + 1e-3 * w * rng.standard_normal(27)
        out = s.collide_node(f)
        assert np.isclose(out.sum(), f.sum(), rtol=1e-14)
        assert np.allclose(out @ c, f @ c, rtol=0, atol=1e-15)
        feq = orc.equilibrium(f.sum(), (f @ c) / f.sum(), 27)
        if coll == "bgk":
            assert np.allclose(out - feq, (1 - 1 / tau) * (f - feq), rtol=0, atol=1e-15)
        if coll == "reg":
            P = lambda g: np.einsum("i,ia,ib->ab", g, c, c)
            assert np.allclose(P(out) - P(feq), (1 - 1 / tau) * (P(f) - P(feq)), atol=1e-15)
            basis = [w] + [w * c[:, a] for a in range(3)] + \
                    [w * c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)]
            B = np.array(basis).T
            coef, *_ = np.linalg.lstsq(B, out, rcond=None)
            assert np.abs(B @ coef - out).max() < 1e-15
        if tau == 1.0:
            assert np.allclose(out, feq, rtol=0, atol=1e-15)


def test_d3q27_streaming_is_a_periodic_shift(orc):
    c, _ = orc.lattice(27)
    nx, ny, nz = 7, 5, 6
    s = orc.OracleSim((nx, ny, nz), lattice=27)
    f = np.random.default_rng(2).random((nx * ny * nz, 27))
    s.set_f(f)
    s.stream_only()
    g = s.get_f()
    for i in range(27):
        rolled = np.roll(f[:, i].reshape(nz, ny, nx), shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        assert np.array_equal(rolled.reshape(-1), g[:, i])


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("trt", 0.8), ("reg", 0.8)])
def test_d3q27_shear_wave_viscosity(orc, coll, tau):
    c, w = orc.lattice(27)
    L = 64
    s = orc.OracleSim((2, L, 2), coll, tau, lattice=27)
    y = (np.arange(s.n) // 2) % L
    u = np.zeros((s.n, 3))
    u[:, 0] = 1e-4 * np.sin(2 * np.pi * y / L)
    s.set_f(feq_field(c, w, 1.0, u))
    amps = []
    for n in (100, 400):
        s.step(n)
        _, uu = s.fields()
        amps.append((uu[:, 0] * np.sin(2 * np.pi * y / L)).sum() * 2 / s.n)
    nu = np.log(amps[0] / amps[1]) / (400 * (2 * np.pi / L) ** 2)
    assert abs(nu / ((tau - 0.5) / 3) - 1) < 0.01


def test_d3q27_couette_between_moving_walls(orc):
    ny, U = 12, 0.01
    s = orc.OracleSim((4, ny, 4), "trt", 0.8, walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0),
                      init="couette", lattice=27)
    m0 = s.mass()
    s.step(300)
    _, u = s.fields()
    y = (np.arange(s.n) // 4) % ny
    fl = (y > 0) & (y < ny - 1)
    ex = -U + 2 * U * (y - 0.5) / (ny - 2)
    assert np.abs(u[fl, 0] - ex[fl]).max() < 1e-10 * U
    assert np.abs(u[fl, 1:]).max() < 1e-14
    assert abs(s.mass() / m0 - 1) < 1e-12


def test_d3q27_moving_particle_conserves_mass_and_momentum(orc):
    s = orc.OracleSim((20, 18, 22), "trt", 0.8, lattice=27)
    q = np.array([0.7, 0.3, -0.5, 0.4])
    pid = s.add_ellipsoid((9.3, 8.7, 10.1), (5.0, 2.5, 2.0), q / np.linalg.norm(q))
    s.set_density(pid, 20.0)
    s.set_velocity(pid, (0.04, -0.03, 0.02), (0.002, -0.003, 0.004))
    m0, P0, mask0 = s.mass(), total_momentum(s, [pid]), s.mask()
    s.step(60)
    assert int((s.mask() != mask0).sum()) > 20
    assert abs(s.mass() / m0 - 1) < 1e-13
    Mu = s.aux(pid)["M"] * np.linalg.norm(s.particle(pid)["U"])
    assert np.abs(total_momentum(s, [pid]) - P0).max() < 1e-12 * Mu


def test_d3q27_links_cover_the_corner_directions(orc):
    """Boundary links: every fluid-to-solid neighbour pair along each of the
    26 directions (brute force over the node map)."""
    L = 16
    s = orc.OracleSim((L, L, L), lattice=27)
    pid = s.add_ellipsoid((7.3, 7.9, 8.2), (4.0, 2.5, 2.0), (0.9, 0.1, -0.3, 0.2) / np.linalg.norm((0.9, 0.1, -0.3, 0.2)))
    c, _ = orc.lattice(27)
    mask = s.mask().reshape(L, L, L)
    want = set()
    for z, y, x in itertools.product(range(L), repeat=3):
        if mask[z, y, x]:
            continue
        for b in range(1, 27):
            xn, yn, zn = (x + c[b, 0]) % L, (y + c[b, 1]) % L, (z + c[b, 2]) % L
            if mask[zn, yn, xn] == pid + 1:
                want.add((x + L * (y + L * z), b))
    site, d = s.links(pid)
    assert set(zip(site.tolist(), d.tolist())) == want
    assert any(b >= 19 for _, b in want)


def test_d3q27_sphere_drag_hasimoto(orc):
    """Sphere R=4, nu=1/6 in a 24^3 box on D3Q27: U 6 pi mu R / F within 5% of
    Hasimoto's periodic-array value (the D3Q19 pin's tolerance)."""
    F, tau, R, L = 1e-4, 1.0, 4.0, 24
    mu = (tau - 0.5) / 3
    s = orc.OracleSim((L, L, L), "bgk", tau, counterforce=True, lattice=27)
    c0 = (L - 1) / 2
    pid = s.add_ellipsoid((c0 + 0.1, c0 + 0.2, c0 + 0.3), (R, R, R), (1, 0, 0, 0))
    s.set_external(pid, (F, 0, 0))
    s.step(800)
    U1 = s.particle(pid)["U"][0]
    s.step(100)
    U = s.particle(pid)["U"][0]
    assert abs(U / U1 - 1) < 2e-4
    assert abs(U * 6 * np.pi * mu * R / F / hasimoto(R / L) - 1) < 0.05
    a = brentq(lambda a: U * 6 * np.pi * mu * a / F - hasimoto(a / L), 2, 8)
    assert abs(a / R - 1) < 0.05


def test_d3q19_and_d3q27_agree_on_a_settling_spheroid(orc):
    """The paper's lattice-independence check (Fig. 3d): the same inclined
    prolate spheroid (a=5, b=c=2.5) under the same force in a 28^3 box moves
    at the same velocity on both lattices, within 0.5% in speed and 0.1 degree
    in direction (measured: 0.17% and 0.01 degree)."""
    L, F = 28, 1e-4
    q = np.array([np.cos(np.pi / 8), 0, np.sin(np.pi / 8), 0])
    U = {}
    for lat in (19, 27):
        s = orc.OracleSim((L, L, L), "trt", 0.8, counterforce=True, lattice=lat)
        pid = s.add_ellipsoid((13.6, 13.3, 13.8), (5.0, 2.5, 2.5), q)
        s.set_external(pid, (0, 0, F))
        s.step(700)
        U[lat] = s.particle(pid)["U"]
    a, b = U[19], U[27]
    assert abs(np.linalg.norm(a) / np.linalg.norm(b) - 1) < 0.005
    cosang = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
    assert np.degrees(np.arccos(min(cosang, 1.0))) < 0.1
