"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Bars: masks and link lists bit-exact (integer work decided by the same FP64
expression); FP64 storage within 1e-9 relative (the oracle keeps full
populations ~w_i while the library keeps deviations ~1e-6, so the oracle's
own representation error is ~1e-16 * 0.05 / 1e-6 ~ 5e-12 relative per value,
and 500 steps accumulate it); FP32 storage within 1e-5 relative on velocity,
force and torque.  Vector comparisons are relative to the vector's norm.
"""
import os
import tempfile

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


def rand_q(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def rel(a, b, floor=0.0):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), floor)


def pair(lb, shape, coll="bgk", tau=1.0, storage="fp64", counterforce=False, walls=False,
         wall_lo=(0, 0, 0), wall_hi=(0, 0, 0), init="rest", max_particles=4, magic=3 / 16, **kw):
    import oracle
    box = lb.make_box(*shape, walls=walls, wall_lo=wall_lo, wall_hi=wall_hi, init=init)
    g = lb.Lattice([box], collision=coll, tau=tau, storage=storage, counterforce=counterforce,
                   max_particles=max_particles, magic=magic, **kw)
    o = oracle.OracleSim(shape, coll, tau, magic=magic, walls=walls, wall_lo=wall_lo,
                         wall_hi=wall_hi, init=init, counterforce=counterforce)
    return g, o


def sorted_links(site, d):
    code = site.astype(np.int64) * 32 + d.astype(np.int64)
    return np.sort(code)


# ----------------------------------------------------------------- geometry --

@pytest.mark.parametrize("seed", range(8))
def test_geometry_bit_exact(lb, seed):
    rng = np.random.default_rng(1000 + seed)
    shape = (20, 17, 23) if seed % 2 else (32, 32, 32)
    g, o = pair(lb, shape)
    centre = rng.random(3) * np.array(shape)
    axes = np.array([5.0, 2.5, 2.0]) * (0.8 + 0.4 * rng.random())
    q = rand_q(rng)
    pg, po = g.add_ellipsoid(centre, axes, q), o.add_ellipsoid(centre, axes, q)
    assert np.array_equal(g.mask(), o.mask())
    sg, so = g.links(pg), o.links(po)
    assert len(sg[0]) == len(so[0]) == g.aux(pg)["nlinks"]
    assert np.array_equal(sorted_links(*sg), sorted_links(*so))


@pytest.mark.parametrize("centre", [(16.0, 16.0, 16.0), (15.5, 15.5, 15.5), (0.0, 31.0, 7.5)])
def test_geometry_exact_surface_nodes(lb, centre):
    """Axis-aligned integer semi-axes put nodes exactly on Q = 1 (strict
    inequality keeps them fluid); a centre on the box edge wraps."""
    g, o = pair(lb, (32, 32, 32))
    pg = g.add_ellipsoid(centre, (4, 2, 2), (1, 0, 0, 0))
    po = o.add_ellipsoid(centre, (4, 2, 2), (1, 0, 0, 0))
    assert np.array_equal(g.mask(), o.mask())
    assert np.array_equal(sorted_links(*g.links(pg)), sorted_links(*o.links(po)))


def test_config1_geometry(lb):
    g, _ = pair(lb, (32, 32, 32))
    pid = g.add_ellipsoid((15.5, 15.5, 15.5), (4, 2, 2), (1, 0, 0, 0))
    assert int((g.mask() == 1).sum()) == 64
    assert g.aux(pid)["nlinks"] == 472


# -------------------------------------------------------------- pure fluid --

@pytest.mark.parametrize("coll,tau,storage,tol", [("bgk", 0.8, "fp64", 1e-12), ("trt", 0.8, "fp64", 1e-12),
                                                  ("reg", 1.2, "fp64", 1e-12), ("trt", 0.8, "fp32", 2e-6)])
def test_couette_fields(lb, coll, tau, storage, tol):
    U = 0.01
    g, o = pair(lb, (6, 12, 5), coll, tau, storage, walls=True, wall_lo=(-U, 0, 0.003),
                wall_hi=(U, 0, -0.002), init="couette")
    g.step(100)
    o.step(100)
    rg, ug = g.fields()
    ro, uo = o.fields()
    assert np.array_equal(rg == 0, ro == 0)
    assert np.abs(ug - uo).max() < tol * U
    assert np.abs(rg - ro).max() < tol


def test_couette_from_rest_fields(lb):
    U = 0.01
    g, o = pair(lb, (4, 10, 4), "bgk", 0.9, "fp64", walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0))
    g.step(200)
    o.step(200)
    assert np.abs(g.fields()[1] - o.fields()[1]).max() < 1e-12 * U


# ------------------------------------------------------------ trajectories --

def compare_particles(g, o, pg, po, tol, start=None, a=4.0):
    """Relative errors with natural scales: torque by |F| a, angular velocity
    by |U| / a (a = largest semi-axis), position and orientation by how far
    they moved since `start` (a zero-by-symmetry quantity is compared against
    the scale of the non-zero ones, not against its own rounding noise)."""
    A, B = g.particle(pg), o.particle(po)
    Fg, Tg = g.force_torque(pg)
    Fo, To = o.force_torque(po)
    nU, nF = np.linalg.norm(B["U"]), np.linalg.norm(Fo)
    start = start or B
    errs = {
        "U": np.abs(A["U"] - B["U"]).max() / nU,
        "W": np.abs(A["W"] - B["W"]).max() / max(np.linalg.norm(B["W"]), nU / a),
        "F": np.abs(Fg - Fo).max() / nF,
        "T": np.abs(Tg - To).max() / max(np.linalg.norm(To), nF * a),
        "x": np.abs(A["x"] - B["x"]).max() / max(np.abs(B["x"] - start["x"]).max(), 1e-300),
        "q": np.abs(A["q"] - B["q"]).max() / max(np.abs(B["q"] - start["q"]).max(), 1e-300),
    }
    for k in ("U", "W", "F", "T"):
        assert errs[k] < tol, (k, errs)
    if start is not B:
        assert errs["x"] < tol and errs["q"] < tol, errs
    print({k: float(f"{v:.3g}") for k, v in errs.items()})
    return errs


def snapshot(o, po):
    return {k: v.copy() for k, v in o.particle(po).items()}


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_config1_trajectory(lb, storage, tol):
    """32^3 BGK tau=1, a=4, b=c=2 centred, F = 1e-4 along x, 500 steps."""
    g, o = pair(lb, (32, 32, 32), "bgk", 1.0, storage, counterforce=True)
    pg = g.add_ellipsoid((15.5, 15.5, 15.5), (4, 2, 2), (1, 0, 0, 0))
    po = o.add_ellipsoid((15.5, 15.5, 15.5), (4, 2, 2), (1, 0, 0, 0))
    g.set_external(pg, (1e-4, 0, 0))
    o.set_external(po, (1e-4, 0, 0))
    x0 = snapshot(o, po)
    x0["q"] = x0["q"] - 1e-6   # orientation does not change: compare at the 1e-6 scale
    for _ in range(5):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, tol, x0)
    # FP64: rounding only; FP32: each stored deviation (~1e-6) carries ~6e-14
    # of rounding, ~3e4 sites x 500 steps of it random-walk to ~1e-12
    assert abs(g.mass() / o.mass() - 1) < (1e-13 if storage == "fp64" else 1e-11)


@pytest.mark.parametrize("axes", [(6, 2, 2), (2, 5, 5), (6, 4, 2)], ids=["prolate", "oblate", "triaxial"])
@pytest.mark.parametrize("storage,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_random_pose_trajectory(lb, storage, tol, axes):
    """Random orientation with force and torque: rotation, dI/dt, quaternion;
    prolate, oblate and triaxial ellipsoids (the method is not restricted to
    prolate spheroids, Sec. IV)."""
    rng = np.random.default_rng(2403054431)
    q = rand_q(rng)
    g, o = pair(lb, (32, 28, 30), "trt", 0.8, storage, counterforce=True)
    c = (15.2, 13.7, 14.9)
    pg, po = g.add_ellipsoid(c, axes, q), o.add_ellipsoid(c, axes, q)
    F, T = (1e-4, -2e-4, 5e-5), (2e-3, 1e-3, -1e-3)
    g.set_external(pg, F, T)
    o.set_external(po, F, T)
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, tol, x0, a=max(axes))


@pytest.mark.parametrize("coll,tau", [("bgk", 1.0), ("trt", 0.8), ("reg", 0.7)])
def test_moving_particle_with_transitions(lb, coll, tau):
    """A heavy, fast ellipsoid crosses many nodes (covered/uncovered)."""
    g, o = pair(lb, (20, 18, 22), coll, tau, "fp64")
    q = np.array([0.7, 0.3, -0.5, 0.4])
    q /= np.linalg.norm(q)
    c = (9.3, 8.7, 10.1)
    pg, po = g.add_ellipsoid(c, (5.0, 2.5, 2.0), q), o.add_ellipsoid(c, (5.0, 2.5, 2.0), q)
    for s, p in ((g, pg), (o, po)):
        s.set_density(p, 20.0)
        s.set_velocity(p, (0.04, -0.03, 0.02), (0.002, -0.003, 0.004))
    m0 = g.mask()
    mass0 = g.mass()
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(20)
        o.step(20)
        compare_particles(g, o, pg, po, 1e-9, x0, a=5.0)
        assert np.array_equal(g.mask(), o.mask())
    assert int((g.mask() != m0).sum()) > 20
    assert abs(g.mass() / mass0 - 1) < 1e-13
    ag, ao = g.aux(pg), o.aux(po)
    assert ag["nlinks"] == ao["nlinks"]
    assert abs(ag["dm"] - ao["dm"]) < 1e-12
    assert np.abs(ag["P"] - ao["P"]).max() < 1e-12


def test_momentum_conservation_gpu(lb):
    g, _ = pair(lb, (20, 18, 22), "bgk", 0.9, "fp64")
    pid = g.add_ellipsoid((9.3, 8.7, 10.1), (5.0, 2.5, 2.0), (0.8, 0.2, -0.4, 0.4) / np.linalg.norm((0.8, 0.2, -0.4, 0.4)))
    g.set_density(pid, 10.0)
    g.set_velocity(pid, (0.03, 0.01, -0.02), (0.001, 0.002, -0.003))

    def total():
        a = g.aux(pid)
        return g.momentum() + a["M"] * g.particle(pid)["U"] + a["P"]
    P0 = total()
    g.step(50)
    assert np.abs(total() - P0).max() < 1e-12 * g.aux(pid)["M"] * 0.03


def test_squirmer_trajectory(lb):
    rng = np.random.default_rng(7)
    q = rand_q(rng)
    g, o = pair(lb, (28, 24, 26), "trt", 1.0, "fp64", magic=3 / 16)
    c = (13.1, 11.9, 12.4)
    pg, po = g.add_ellipsoid(c, (5, 2.5, 2.5), q), o.add_ellipsoid(c, (5, 2.5, 2.5), q)
    g.set_squirmer(pg, 1e-3, 2e-3)
    o.set_squirmer(po, 1e-3, 2e-3)
    x0 = snapshot(o, po)
    for _ in range(2):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, 1e-9, x0, a=5.0)


def test_particle_between_moving_walls(lb):
    """Jeffery set-up: neutrally buoyant spheroid in Couette flow."""
    U = 0.01
    g, o = pair(lb, (24, 26, 20), "bgk", 0.8, "fp64", walls=True, wall_lo=(-U, 0, 0), wall_hi=(U, 0, 0),
                init="couette")
    q = np.array([0.9, 0.1, 0.3, 0.2])
    q /= np.linalg.norm(q)
    c = (11.6, 12.4, 9.7)
    pg, po = g.add_ellipsoid(c, (6, 3, 3), q), o.add_ellipsoid(c, (6, 3, 3), q)
    x0 = snapshot(o, po)
    for _ in range(3):
        g.step(100)
        o.step(100)
        compare_particles(g, o, pg, po, 1e-9, x0, a=6.0)
    assert np.array_equal(g.mask(), o.mask())


def test_two_particles(lb):
    g, o = pair(lb, (24, 20, 20), "bgk", 0.9, "fp64")
    specs = [((6.2, 10.1, 9.8), (4, 2, 2), (1, 0, 0, 0), (0.02, 0.01, 0.0), (0, 0, 0.003)),
             ((17.7, 9.4, 10.3), (3.5, 2.5, 2), (0.8, 0.0, 0.6, 0.0), (-0.02, 0.0, 0.01), (0.002, 0, 0))]
    ids = []
    for c, a, q, U, W in specs:
        pg, po = g.add_ellipsoid(c, a, q), o.add_ellipsoid(c, a, q)
        for s, p in ((g, pg), (o, po)):
            s.set_density(p, 5.0)
            s.set_velocity(p, U, W)
        ids.append((pg, po, snapshot(o, po)))
    g.step(40)
    o.step(40)
    for pg, po, x0 in ids:
        compare_particles(g, o, pg, po, 1e-9, x0)
    assert np.array_equal(g.mask(), o.mask())


@pytest.mark.parametrize("variant", ["0", "12"], ids=["pull", "in-place"])
def test_two_particles_closing_to_one_node_gap(lb, variant):
    """Two particles pulled towards each other until a single fluid node
    separates them (the oracle reports an overlap at step 330; the run stops
    at 318).  When one of them covers or uncovers a node beside the other, the
    other's link list changes although none of its own nodes did: the node map
    of step t+1 is complete before any link list is rebuilt (Appendix A,
    steps 8-9).  Masks and link lists equal the oracle's bit for bit after
    every step; such link changes happen (counted on the oracle, so a remap
    that kept stale links would fail here); trajectories within the FP64 bar."""
    os.environ["LBELL_K1_VARIANT"] = variant
    try:
        g, o = pair(lb, (40, 20, 22), "bgk", 0.9, "fp64")
    finally:
        del os.environ["LBELL_K1_VARIANT"]
    specs = [((14.6, 9.6, 10.8), (5.0, 3.0, 2.5), (0.95, 0.1, 0.2, 0.2), 1.0),
             ((24.5, 10.2, 11.1), (4.5, 3.5, 2.5), (0.9, -0.2, 0.1, 0.35), -1.0)]
    ids = []
    for c, ax, q, sgn in specs:
        q = np.array(q) / np.linalg.norm(q)
        pg, po = g.add_ellipsoid(c, ax, q), o.add_ellipsoid(c, ax, q)
        for s, p in ((g, pg), (o, po)):
            s.set_external(p, (0.06 * sgn, 5e-4 * sgn, 0.0), (0.0, 0.0, 2e-3 * sgn))
        ids.append((pg, po, snapshot(o, po)))
    (ga, oa, _), (gb, ob, _) = ids

    def linkset(sim, p):
        return sorted_links(*sim.links(p))

    m_prev = o.mask()
    prev = [linkset(o, oa), linkset(o, ob)]
    foreign = 0
    for step in range(318):
        g.step(1)
        o.step(1)
        m = o.mask()
        assert np.array_equal(g.mask(), m), step
        cur = [linkset(o, oa), linkset(o, ob)]
        for k, (pg, po) in enumerate(((ga, oa), (gb, ob))):
            assert np.array_equal(linkset(g, pg), cur[k]), (step, k)
            own_changed = ((m_prev == po + 1) != (m == po + 1)).any()
            if not own_changed and not np.array_equal(cur[k], prev[k]):
                foreign += 1
        m_prev, prev = m, cur
    assert o.overlaps() == 0
    print("link lists changed by the other particle:", foreign)
    assert foreign >= 3
    for pg, po, x0 in ids:
        compare_particles(g, o, pg, po, 1e-9, x0, a=5.0)


@pytest.mark.parametrize("axis", [0, 2], ids=["axial", "transverse"])
def test_torque_driven_spin(lb, axis):
    """A torque-driven r = 2 spheroid spinning up about / across its axis
    (the run the oracle's rotational-resistance pin checks against X^C and
    Y^C), 400 steps in 32^3: the GPU at the FP64 bar."""
    g, o = pair(lb, (32, 32, 32), "bgk", 1.0, "fp64")
    T = [0.0, 0.0, 0.0]
    T[axis] = 1e-3
    pg = g.add_ellipsoid((15.63, 15.29, 15.57), (6.0, 3.0, 3.0), (1, 0, 0, 0))
    po = o.add_ellipsoid((15.63, 15.29, 15.57), (6.0, 3.0, 3.0), (1, 0, 0, 0))
    g.set_external(pg, (0, 0, 0), T)
    o.set_external(po, (0, 0, 0), T)
    g.step(400)
    o.step(400)
    A, B = g.particle(pg), o.particle(po)
    nW = np.linalg.norm(B["W"])
    assert nW > 1e-6
    assert np.abs(A["W"] - B["W"]).max() / nW < 1e-9
    Tg = g.force_torque(pg)[1]
    To = o.force_torque(po)[1]
    assert np.abs(Tg - To).max() / np.linalg.norm(To) < 1e-9


# ----------------------------------------------------------------- batching --

def test_batch_matches_single_boxes_bitwise(lb):
    """Boxes of uneven size stepped in one launch give the same bits as each
    box alone, and match the oracle."""
    import oracle
    specs = [((24, 20, 28), (11.2, 9.7, 13.1), (5, 2.5, 2.5), (0.9, 0.1, -0.2, 0.3)),
             ((17, 19, 21), (8.4, 9.1, 10.3), (4, 2, 2), (0.6, -0.5, 0.4, 0.2))]
    boxes = [lb.make_box(*s[0]) for s in specs]
    batch = lb.Lattice(boxes, collision="trt", tau=0.8, storage="fp32", counterforce=True, max_particles=2)
    singles = []
    for b, (shape, c, a, q) in enumerate(specs):
        q = np.array(q) / np.linalg.norm(q)
        pid = batch.add_ellipsoid(c, a, q, box=b)
        batch.set_external(pid, (1e-4, 2e-5 * (b + 1), 0), (0, 0, 1e-4))
        s = lb.Lattice([lb.make_box(*shape)], collision="trt", tau=0.8, storage="fp32", counterforce=True)
        sp = s.add_ellipsoid(c, a, q)
        s.set_external(sp, (1e-4, 2e-5 * (b + 1), 0), (0, 0, 1e-4))
        singles.append(s)
    batch.step(60)
    for b, s in enumerate(singles):
        s.step(60)
        pb, ps = batch.particle(b), s.particle(0)
        for k in pb:
            assert np.array_equal(pb[k], ps[k]), k
        assert np.array_equal(batch.fields(b)[1], s.fields(0)[1])
    o = oracle.OracleSim(specs[1][0], "trt", 0.8, counterforce=True)
    q = np.array(specs[1][3]) / np.linalg.norm(specs[1][3])
    po = o.add_ellipsoid(specs[1][1], specs[1][2], q)
    o.set_external(po, (1e-4, 4e-5, 0), (0, 0, 1e-4))
    o.step(60)
    assert rel(batch.particle(1)["U"], o.particle(po)["U"]) < 1e-5


# ------------------------------------------------------ systems behaviour --

def test_checkpoint_roundtrip_bitwise(lb):
    def make():
        g, _ = pair(lb, (20, 18, 22), "trt", 0.8, "fp32", counterforce=True)
        p = g.add_ellipsoid((9.3, 8.7, 10.1), (5.0, 2.5, 2.0), (1, 0, 0, 0))
        g.set_external(p, (1e-4, 0, 5e-5), (0, 1e-4, 0))
        return g, p
    a, pa = make()
    a.step(30)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.save(path)
        a.step(30)
        b, pb = make()
        b.load(path)
        assert b.step_count() == 30
        b.step(30)
    for k, v in a.particle(pa).items():
        assert np.array_equal(v, b.particle(pb)[k]), k
    assert np.array_equal(a.fields()[1], b.fields()[1])


def test_checkpoint_of_another_version_is_rejected(lb):
    """The header's format version (the int after the 8-byte magic) must be
    this library's; a file claiming another is refused with LB_EINVAL and the
    context keeps running."""
    import struct
    g, _ = pair(lb, (20, 18, 22), "trt", 0.8, "fp32", counterforce=True)
    p = g.add_ellipsoid((9.3, 8.7, 10.1), (5.0, 2.5, 2.0), (1, 0, 0, 0))
    g.step(5)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        g.save(path)
        raw = bytearray(open(path, "rb").read())
        (ver,) = struct.unpack_from("<i", raw, 8)
        struct.pack_into("<i", raw, 8, ver - 1)
        open(path, "wb").write(bytes(raw))
        with pytest.raises(lb.LBError) as e:
            g.load(path)
        assert lb.STATUS[e.value.status] == "LB_EINVAL"
    g.step(5)
    assert g.step_count() == 10 and np.isfinite(g.particle(p)["U"]).all()


def test_nonfinite_watchdog(lb):
    g, _ = pair(lb, (16, 16, 16), "bgk", 1.0, "fp32")
    assert g.nonfinite() == 0
    g.poke(0, 5 + 16 * (6 + 16 * 7), 3, float("nan"))
    assert g.nonfinite() >= 1


def test_overlap_is_rejected(lb):
    g, _ = pair(lb, (24, 24, 24), "bgk", 1.0, "fp32")
    g.add_ellipsoid((12, 12, 12), (5, 2.5, 2.5), (1, 0, 0, 0))
    with pytest.raises(lb.LBError) as e:
        g.add_ellipsoid((14, 12, 12), (5, 2.5, 2.5), (1, 0, 0, 0))
    assert e.value.status == -5
    # the failed particle left nothing behind
    assert int((g.mask() == 2).sum()) == 0
    assert g.add_ellipsoid((12, 12, 2.5), (4, 2, 2), (1, 0, 0, 0)) == 1


def test_invalid_particle_arguments(lb):
    g, _ = pair(lb, (16, 16, 16), "bgk", 1.0, "fp32")
    with pytest.raises(lb.LBError):
        g.add_ellipsoid((8, 8, 8), (7.5, 2, 2), (1, 0, 0, 0))      # does not fit
    with pytest.raises(lb.LBError):
        g.add_ellipsoid((8, 8, 8), (4, 2, 2), (1, 0.1, 0, 0))      # not unit
    with pytest.raises(lb.LBError):
        g.add_ellipsoid((8, 8, 8), (4, -2, 2), (1, 0, 0, 0))


# ------------------------------------------------- collide-stream variants --

def _variant_lattice(lb, variant, shape, storage, walls=False):
    os.environ["LBELL_K1_VARIANT"] = str(variant)
    try:
        U = 0.01
        box = lb.make_box(*shape, walls=walls, wall_lo=(-U, 0, 0) if walls else (0, 0, 0),
                          wall_hi=(U, 0, 0) if walls else (0, 0, 0), init="couette" if walls else "rest")
        g = lb.Lattice([box], collision="trt", tau=0.8, storage=storage, counterforce=not walls)
    finally:
        del os.environ["LBELL_K1_VARIANT"]
    q = np.array([0.8, 0.3, -0.4, 0.33])
    p = g.add_ellipsoid((31.3, shape[1] / 2 - 0.4, shape[2] / 2 + 0.2), (6, 2.5, 2), q / np.linalg.norm(q))
    if not walls:
        g.set_external(p, (1e-4, -5e-5, 2e-4), (1e-3, 0, 0))
    return g, p


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("nx,walls", [(64, False), (128, False), (64, True)])
def test_row_wave_variants_bitwise(lb, storage, nx, walls):
    """The row-wave kernel (with and without non-temporal stores) produces the
    same bits as the generic tile kernel."""
    shape = (nx, 22, 18)
    runs = []
    for v in (0, 1, 2):
        g, p = _variant_lattice(lb, v, shape, storage, walls)
        g.step(25)
        runs.append((g.particle(p), g.fields()[1]))
    for pr, u in runs[1:]:
        for k in pr:
            assert np.array_equal(pr[k], runs[0][0][k]), k
        assert np.array_equal(u, runs[0][1])


def test_row_wave_matches_oracle(lb):
    import oracle
    g, p = _variant_lattice(lb, 1, (64, 22, 18), "fp64")
    o = oracle.OracleSim((64, 22, 18), "trt", 0.8, counterforce=True)
    q = np.array([0.8, 0.3, -0.4, 0.33])
    po = o.add_ellipsoid((31.3, 22 / 2 - 0.4, 18 / 2 + 0.2), (6, 2.5, 2), q / np.linalg.norm(q))
    o.set_external(po, (1e-4, -5e-5, 2e-4), (1e-3, 0, 0))
    x0 = snapshot(o, po)
    g.step(100)
    o.step(100)
    compare_particles(g, o, p, po, 1e-9, x0, a=6.0)


def test_autotune_keeps_state(lb):
    g, p = _variant_lattice(lb, 1, (128, 20, 16), "fp32")
    h, hp = _variant_lattice(lb, 1, (128, 20, 16), "fp32")
    g.step(10)
    h.step(10)
    t0 = g.step_count()
    v, ms = g.autotune(5)
    assert v in range(16) and ms > 0
    h.step(g.step_count() - t0)  # the tuner's timed steps are ordinary steps
    g.step(10)
    h.step(10)
    for k, val in g.particle(p).items():
        assert np.array_equal(val, h.particle(hp)[k]), k


def _moving_lattice(lb, overlap, shape, storage, nboxes=1):
    os.environ["LBELL_OVERLAP"] = str(overlap)
    try:
        g = lb.Lattice([lb.make_box(*shape)] * nboxes, collision="bgk", tau=0.9, storage=storage,
                       max_particles=2 * nboxes)
    finally:
        del os.environ["LBELL_OVERLAP"]
    ids = []
    for b in range(nboxes):
        q = np.array([0.7, 0.3, -0.5, 0.4])
        p = g.add_ellipsoid((shape[0] / 2 + 0.3, shape[1] / 2 - 0.2, shape[2] / 2 + 0.1), (5.0, 2.5, 2.0),
                            q / np.linalg.norm(q), box=b)
        g.set_density(p, 20.0)
        g.set_velocity(p, (0.04, -0.03, 0.02), (0.002, -0.003, 0.004))
        ids.append(p)
    return g, ids


@pytest.mark.parametrize("shape,storage,nboxes", [((128, 24, 20), "fp32", 1), ((64, 20, 22), "fp64", 1),
                                                  ((20, 18, 22), "fp32", 3)])
def test_overlapped_schedule_matches_serial(lb, shape, storage, nboxes):
    """Far blocks on the caller's stream, near blocks + particles on the second
    stream: the same bits as the one-stream schedule, for a fast particle
    that crosses nodes every few steps."""
    runs = []
    for ov in (0, 1):
        g, ids = _moving_lattice(lb, ov, shape, storage, nboxes)
        for _ in range(4):
            g.step(15)
        runs.append((g, ids))
    (a, ia), (b, ib) = runs
    for pa, pb in zip(ia, ib):
        for k, v in a.particle(pa).items():
            assert np.array_equal(v, b.particle(pb)[k]), k
    for bx in range(nboxes):
        assert np.array_equal(a.fields(bx)[1], b.fields(bx)[1])
        assert np.array_equal(a.mask(bx), b.mask(bx))


def test_checkpoint_reload_into_advanced_context(lb):
    """Loading an earlier checkpoint into a context that has run further
    (step counter moves back) reproduces the uninterrupted run bit for bit."""
    def make():
        g = lb.Lattice([lb.make_box(128, 20, 18)], collision="trt", tau=0.8, storage="fp32")
        q = np.array([0.8, 0.2, 0.3, -0.4])
        p = g.add_ellipsoid((60.2, 9.7, 8.9), (5.0, 2.5, 2.0), q / np.linalg.norm(q))
        g.set_density(p, 20.0)
        g.set_velocity(p, (0.04, -0.02, 0.01), (0.001, 0.002, -0.003))
        return g, p
    a, pa = make()
    b, pb = make()
    b.step(60)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        a.step(30)
        a.save(path)
        a.step(30)
        b.load(path)                    # b was at step 60
    b.step(30)
    for k, v in a.particle(pa).items():
        assert np.array_equal(v, b.particle(pb)[k]), k
    assert np.array_equal(a.fields()[1], b.fields()[1])


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_fused_particle_kernel_matches_two_kernels(lb, storage):
    """One work-group doing solve + remap (boxes with one particle) gives the
    same bits as the two-kernel path."""
    runs = []
    for fused in ("1", "0"):
        os.environ["LBELL_FUSED"] = fused
        try:
            g, ids = _moving_lattice(lb, 0, (20, 18, 22), storage, nboxes=2)
        finally:
            del os.environ["LBELL_FUSED"]
        g.step(60)
        runs.append((g, ids))
    (a, ia), (b, ib) = runs
    for pa, pb in zip(ia, ib):
        for k, v in a.particle(pa).items():
            assert np.array_equal(v, b.particle(pb)[k]), k
        Fa, Ta = a.force_torque(pa)
        Fb, Tb = b.force_torque(pb)
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
    for bx in range(2):
        assert np.array_equal(a.fields(bx)[1], b.fields(bx)[1])
