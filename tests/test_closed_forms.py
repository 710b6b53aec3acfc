"""Pins of the host-side closed forms the control start and the studies use
(no GPU): Oberbeck's ellipsoid resistances by quadrature against the
Kim-Karrila prolate-spheroid functions (two independent derivations), the
sphere's Stokes values, the thin-disk limits, and axis permutation."""
import math

import numpy as np
import pytest

from paper_2403_05443_amd import runner


@pytest.mark.parametrize("r", [1.0, 1.2, 2.0, 3.0, 5.0])
def test_oberbeck_matches_kim_karrila_for_prolate(r):
    mu, b = 0.1, 2.5
    a = r * b
    tr, ro = runner.ellipsoid_resistance((a, b, b), mu)
    XA, YA, XC, YC = runner.resistance(r)
    assert np.allclose(tr / (6 * math.pi * mu * a), [XA, YA, YA], rtol=1e-12, atol=0)
    assert np.allclose(ro / (8 * math.pi * mu * a ** 3), [XC, YC, YC], rtol=1e-12, atol=0)


def test_sphere_stokes():
    tr, ro = runner.ellipsoid_resistance((3.0, 3.0, 3.0), 0.2)
    assert np.allclose(tr, 6 * math.pi * 0.2 * 3.0, rtol=1e-13)
    assert np.allclose(ro, 8 * math.pi * 0.2 * 27.0, rtol=1e-13)


def test_thin_disk_limits():
    """a -> 0: broadside translation 16 mu b, edgewise 32 mu b / 3, spin about
    the axis 32 mu b^3 / 3 (the flat-disk results)."""
    tr, ro = runner.ellipsoid_resistance((1e-4, 1.0, 1.0), 1.0, n=2000)
    assert abs(tr[0] / 16 - 1) < 1e-3
    assert abs(tr[1] / (32 / 3) - 1) < 1e-3 and abs(tr[2] / (32 / 3) - 1) < 1e-3
    assert abs(ro[0] / (32 / 3) - 1) < 1e-3


def test_axis_permutation():
    tr, ro = runner.ellipsoid_resistance((6.0, 4.0, 2.0), 0.1)
    tp, rp = runner.ellipsoid_resistance((2.0, 6.0, 4.0), 0.1)
    assert np.allclose(tp, tr[[2, 0, 1]], rtol=1e-12) and np.allclose(rp, ro[[2, 0, 1]], rtol=1e-12)
    # a longer axis is the cheaper direction to move along
    assert tr[0] < tr[1] < tr[2]
