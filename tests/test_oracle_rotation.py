"""Pins of the oracle's three treatments of the inertia in the rotational
equation (Sec. II.D): eq. Tdiscrete with the analytic dI/dt of eq. Irotdiff
(mode 0), with the finite difference (I(t) - I(t - dt)) / dt (mode 1), and
the predictor-corrector for I(t + dt) (mode 2, reading R21).  Each step's
rotational balance is rebuilt from the states before and after the step and
the reported hydrodynamic torque, with the body inertia from its closed form
(not from the oracle):
  mode 0:  (I(t) + [W]x I(t) - I(t) [W]x) W' - I(t) W = T + T_ext
  mode 1:  (2 I(t) - I(t - dt)) W' - I(t) W = T + T_ext
  mode 2:  I(t + dt) W' - I(t) W = T + T_ext, with I(t + dt) from the
           predicted orientation, so the final orientation reproduces it
           only up to the change of the mean rate between predictor and
           corrector.
Also: for a sphere all three modes coincide, and for a slowly rotating
spheroid they agree closely (the paper saw no difference between 0 and 1)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def lab_inertia(q, M, axes):
    a, b, c = axes
    Ib = np.diag([M * (b * b + c * c) / 5, M * (a * a + c * c) / 5, M * (a * a + b * b) / 5])
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R @ Ib @ R.T


def cross_mat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


AXES = (5.0, 2.5, 2.0)
TEXT = np.array([2e-3, -1e-3, 1.5e-3])


def run(orc, mode, axes=AXES, steps=40):
    s = orc.OracleSim((22, 20, 24), "trt", 0.8, rotation=mode)
    q = np.array([0.8, 0.2, -0.4, 0.4])
    q /= np.linalg.norm(q)
    pid = s.add_ellipsoid((10.6, 9.3, 11.8), axes, q)
    s.set_external(pid, (0, 0, 0), TEXT)
    s.set_velocity(pid, (0, 0, 0), (0.004, -0.003, 0.002))
    hist = []
    for _ in range(steps):
        before = s.particle(pid)
        s.step(1)
        after = s.particle(pid)
        hist.append((before, after, s.force_torque(pid)[1]))
    return s, pid, hist


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_rotational_balance(orc, mode):
    s, pid, hist = run(orc, mode)
    M = s.aux(pid)["M"]
    worst = 0.0
    for k, (b, a, T) in enumerate(hist):
        I0 = lab_inertia(b["q"], M, AXES)
        W0, W1 = b["W"], a["W"]
        if mode == 0:
            Wx = cross_mat(W0)
            lhs = (I0 + Wx @ I0 - I0 @ Wx) @ W1 - I0 @ W0
        elif mode == 1:
            Ip = lab_inertia(hist[k - 1][0]["q"], M, AXES) if k > 0 else I0
            lhs = (2 * I0 - Ip) @ W1 - I0 @ W0
        else:
            lhs = lab_inertia(a["q"], M, AXES) @ W1 - I0 @ W0
        rhs = T + TEXT
        worst = max(worst, np.abs(lhs - rhs).max() / np.abs(rhs).max())
    print("mode", mode, "worst relative residual", worst)
    # mode 2: 1.4e-7 measured; modes 0 and 1 miss this balance by 3e-4 and
    # 2e-3, so the bound tells the predictor-corrector from the others.
    assert worst < (1e-10 if mode < 2 else 1e-5)


def test_modes_coincide_for_a_sphere(orc):
    runs = [run(orc, m, axes=(3.0, 3.0, 3.0), steps=30) for m in (0, 1, 2)]
    ref = runs[0][0].particle(runs[0][1])
    for s, pid, _ in runs[1:]:
        p = s.particle(pid)
        for k in ("U", "W", "q"):
            assert np.allclose(p[k], ref[k], rtol=0, atol=1e-10 * np.abs(ref[k]).max()), k


def test_modes_agree_for_a_slow_spheroid(orc):
    runs = [run(orc, m, steps=60) for m in (0, 1, 2)]
    W0 = runs[0][0].particle(runs[0][1])["W"]
    for s, pid, _ in runs[1:]:
        W = s.particle(pid)["W"]
        print(np.abs(W - W0).max() / np.abs(W0).max())
        assert np.abs(W - W0).max() < 2e-2 * np.abs(W0).max()
