"""The rule by which the remap skips testing a particle's window (no node can
have changed side since the last test), checked as a property of the
geometry on the CPU: for random ellipsoids, reference poses and small rigid
motions, whenever the rule allows a skip, brute force over every node near
the body finds the same inside/outside state as at the reference pose.

The rule: at the reference pose every node x of the window [floor(x_c - h) - 2,
floor(x_c + h) + 1] (h the half-extents of the bounding box) has
2 |Q - 1| / (Q + 3) >= m (a lower bound of |sqrt(Q) - 1|); after the centre
moved by dx and the body turned by th, skip iff
(dx + 2 sin(th/2) rho) < m min(a, b, c) and dx + 2 sin(th/2) max(a, b, c) < 1/2,
rho the largest |x - x_c| over the window."""
import numpy as np
from scipy.spatial.transform import Rotation


def quad(nodes, c, R, axes):
    y = (nodes - c) @ R            # body coordinates R^T (x - c), row-wise
    return ((y / axes) ** 2).sum(axis=1)


def window(c, R, axes):
    h = np.sqrt(((R * axes) ** 2).sum(axis=1))
    lo = np.floor(c - h - 1e-9) - 1
    hi = np.floor(c + h + 1e-9) + 1
    g = np.stack(np.meshgrid(*[np.arange(l, u + 1) for l, u in zip(lo, hi)], indexing="ij"), -1).reshape(-1, 3)
    return g


def test_skip_rule_never_misses_a_change():
    rng = np.random.default_rng(240305)
    skips = changes_seen = 0
    for trial in range(400):
        axes = np.sort(rng.uniform(1.5, 6.0, 3))[::-1]
        c = rng.uniform(10, 11, 3)
        R = Rotation.random(random_state=rng).as_matrix()
        win = window(c, R, axes)
        Qw = quad(win, c, R, axes)
        m = (2 * np.abs(Qw - 1) / (Qw + 3)).min()
        rho = np.linalg.norm(win - c, axis=1).max()
        # every node that could matter: a generous cube around the body
        big = window(c, R, axes + 3)
        inside0 = quad(big, c, R, axes) < 1
        for _ in range(20):
            scale = 10.0 ** rng.uniform(-4, -0.5)
            dxv = rng.standard_normal(3) * scale
            th = abs(rng.standard_normal()) * scale / max(axes)
            ax = rng.standard_normal(3)
            dR = Rotation.from_rotvec(th * ax / np.linalg.norm(ax)).as_matrix()
            c1, R1 = c + dxv, dR @ R
            dx, sh = np.linalg.norm(dxv), np.sin(th / 2)
            skip = (dx + 2 * sh * rho) < m * axes.min() and dx + 2 * sh * axes.max() < 0.5
            inside1 = quad(big, c1, R1, axes) < 1
            if skip:
                skips += 1
                assert np.array_equal(inside0, inside1), (trial, dx, th)
            elif not np.array_equal(inside0, inside1):
                changes_seen += 1
    print("skips", skips, "motions with a change", changes_seen)
    assert skips > 1000 and changes_seen > 100
