"""Pins of the oracle's geometry (Sec. II.B, eq. ellipsoidsurface) and drag
matrices (eqs. drag1-drag4) against an independent formulation: the matrix A
of the paper built from scipy's rotation matrix, brute-force link search with
np.roll, and hand-derived counts for the axis-aligned case."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def quadratic_form(shape, centre, axes, quat):
    """(x - x_c)^T A (x - x_c) at every node, A = R diag(1/a^2, 1/b^2, 1/c^2) R^T,
    minimum-image separations; returns array indexed by site."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.stack([x.ravel() - centre[0], y.ravel() - centre[1], z.ravel() - centre[2]], 1)
    n = np.array(shape, dtype=float)
    d = d - n * np.round(d / n)
    q = np.asarray(quat, float) / np.linalg.norm(quat)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    A = R @ np.diag(1.0 / np.asarray(axes, float) ** 2) @ R.T
    return np.einsum("ni,ij,nj->n", d, A, d)


def brute_links(shape, solid, c):
    nx, ny, nz = shape
    S = solid.reshape(nz, ny, nx)
    out = set()
    for b in range(1, 19):
        nb = np.roll(S, shift=(-c[b, 2], -c[b, 1], -c[b, 0]), axis=(0, 1, 2))
        sites = np.nonzero((~S & nb).ravel())[0]
        out.update((int(s), b) for s in sites)
    return out


def random_pose(rng, shape):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    centre = rng.random(3) * np.array(shape)
    return centre, q


@pytest.mark.parametrize("seed", range(6))
def test_mask_and_links_match_independent_form(orc, seed):
    """Solid iff Q < 1 (strict, reading of 'inside'); boundary links are every
    (fluid x, b) with x + c_b solid.  Nodes within 1e-9 of the surface are
    skipped in the mask comparison (rounding may legitimately differ there)."""
    c, _ = orc.lattice()
    rng = np.random.default_rng(100 + seed)
    shape = (20, 17, 23)
    centre, q = random_pose(rng, shape)
    axes = np.array([5.0, 2.5, 2.0]) * (0.8 + 0.4 * rng.random())
    s = orc.OracleSim(shape)
    pid = s.add_ellipsoid(centre, axes, q)
    m = s.mask()
    Q = quadratic_form(shape, centre, axes, q)
    solid = m == pid + 1
    sure = np.abs(Q - 1) > 1e-9
    assert np.array_equal(solid[sure], (Q < 1)[sure])
    site, d = s.links(pid)
    got = set(zip(site.tolist(), d.tolist()))
    assert got == brute_links(shape, solid, c)
    assert len(got) == s.aux(pid)["nlinks"]


def test_config1_counts_and_zeta(orc):
    """a=4, b=c=2 centred at 15.5^3 of a 32^3 box: hand-derived counts."""
    g = json.load(open(os.path.join(GOLD, "c1_geometry.json")))
    c, _ = orc.lattice()
    s = orc.OracleSim((32, 32, 32))
    pid = s.add_ellipsoid((15.5, 15.5, 15.5), (4, 2, 2), (1, 0, 0, 0))
    assert int((s.mask() == 1).sum()) == g["solid_nodes"]
    site, d = s.links(pid)
    assert len(site) == g["links"]
    assert int((d <= 6).sum()) == g["face_links"]
    diag = [int(((d > 6) & (c[d, k] != 0)).sum()) for k in range(3)]
    assert diag == g["diagonal_links_per_axis"]
    z = s.zeta(pid)
    assert np.allclose(np.diag(z[:3, :3]), g["zeta_FU_diag"], rtol=1e-14)
    assert np.abs(z[:3, :3] - np.diag(np.diag(z[:3, :3]))).max() < 1e-13
    # symmetric placement: no translation-rotation coupling
    assert np.abs(z[:3, 3:]).max() < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_zeta_structure(orc, seed):
    """zeta_TU = zeta_FW^T (eqs. drag2, drag3 are transposes); the 6x6 drag
    matrix is symmetric positive semi-definite; sum_b w_b c_b = 0 and
    sum_b w_b (x_b - x_c) x c_b = 0 over a closed link set."""
    c, w = orc.lattice()
    rng = np.random.default_rng(seed)
    shape = (24, 24, 24)
    centre, q = random_pose(rng, shape)
    s = orc.OracleSim(shape)
    pid = s.add_ellipsoid(centre, (6.0, 2.0, 3.0), q)
    z = s.zeta(pid)
    assert np.allclose(z[3:, :3], z[:3, 3:].T, rtol=0, atol=1e-12)
    assert np.allclose(z, z.T, rtol=0, atol=1e-11)
    assert np.linalg.eigvalsh(z).min() > -1e-9
    site, d = s.links(pid)
    assert np.abs((w[d][:, None] * c[d]).sum(0)).max() < 1e-12
    # the translational block is an integer combination: 6*w = 1/3 or 1/6
    zfu = z[:3, :3] * 6
    assert np.allclose(zfu, np.round(zfu), atol=1e-10)


def test_wrapped_particle_matches_unwrapped(orc):
    """An ellipsoid straddling the periodic boundary has the same shape (mask
    shifted) as the same ellipsoid in the middle of the box."""
    shape = (16, 16, 16)
    q = np.array([0.9, 0.2, -0.3, 0.25])
    q /= np.linalg.norm(q)
    s1 = orc.OracleSim(shape)
    s1.add_ellipsoid((8.3, 8.1, 7.7), (4.5, 2.5, 2.0), q)
    s2 = orc.OracleSim(shape)
    s2.add_ellipsoid((8.3 - 8, 8.1 + 8, 7.7 - 8), (4.5, 2.5, 2.0), q)
    m1 = (s1.mask() == 1).reshape(16, 16, 16)
    m2 = (s2.mask() == 1).reshape(16, 16, 16)
    assert np.array_equal(np.roll(m1, shift=(-8, 8, -8), axis=(0, 1, 2)), m2)
    assert s1.aux(0)["nlinks"] == s2.aux(0)["nlinks"]
