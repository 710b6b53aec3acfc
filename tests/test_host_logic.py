"""Host-side logic of the learned part and the steps-to-steady metric (no
GPU): the augmentation maps samples of a spheroid's linear response to
samples of the same response, the seeded shuffle is a permutation, and the
steps-to-tolerance count follows its definition on hand-built trajectories."""
import math

import numpy as np

from paper_2403_05443_amd import runner


def _spheroid_response(X, m=(0.8, 0.6), k=(0.3, 0.9)):
    """Normalised body-frame response of a body symmetric about its x axis:
    U = diag(m1, m2, m2) F, Omega = diag(k1, k2, k2) T (the form the
    mobility of a spheroid takes in its body frame)."""
    Y = np.zeros((len(X), 6))
    Y[:, 0:3] = X[:, 2:5] * np.array([m[0], m[1], m[1]])
    Y[:, 3:6] = X[:, 5:8] * np.array([k[0], k[1], k[1]])
    return Y


def test_augment_keeps_the_linear_response():
    g = np.random.default_rng(5)
    X = g.standard_normal((7, 8))
    Y = _spheroid_response(X)
    Xa, Ya = runner.augment(X, Y)
    assert len(Xa) == 32 * len(X)  # 8 rotations x head-tail x load reversal
    assert np.allclose(Xa[:, 0:2], np.tile(X[:, 0:2], (32, 1)))  # shape inputs unchanged
    assert np.allclose(Ya, _spheroid_response(Xa), atol=1e-14)
    # a response that is not axisymmetric is not mapped onto itself: the
    # check above would catch rotations about another axis
    Yb = X[:, 2:8] * np.array([0.8, 0.6, 0.4, 0.3, 0.9, 0.5])
    Xb, Yb2 = runner.augment(X, Yb)
    assert not np.allclose(Yb2, Xb[:, 2:8] * np.array([0.8, 0.6, 0.4, 0.3, 0.9, 0.5]), atol=1e-6)
    # load reversal alone
    Xn, Yn = runner.augment(X, Y, nrot=1, flip=False, negate=True)
    assert np.allclose(Xn[len(X):, 2:], -X[:, 2:]) and np.allclose(Yn[len(X):], -Y)


def test_shuffle_is_a_seeded_permutation():
    X = np.arange(40, dtype=float).reshape(20, 2)
    Y = np.arange(20, dtype=float)[:, None]
    A, B = runner.shuffle(X, Y, 7)
    A2, _ = runner.shuffle(X, Y, 7)
    A3, _ = runner.shuffle(X, Y, 8)
    assert sorted(A[:, 0].tolist()) == X[:, 0].tolist() and np.array_equal(A[:, 0] / 2, B[:, 0])
    assert np.array_equal(A, A2) and not np.array_equal(A, A3)


def test_steps_to_tolerance_definition():
    times = np.arange(1, 9) * 25
    Uinf = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 1.0]])
    U = np.repeat(Uinf[None], 8, axis=0).copy()
    U[:3, 0, 0] = [0.5, 0.9, 0.999]      # particle 0: within 0.5 % from the 3rd sample on
    U[5, 1, 1] = 2.02                    # particle 1: leaves the band at the 6th sample
    U[:, 2, 2] = 1.1                     # particle 2: never within
    n = runner.steps_to_tolerance(times, U, Uinf, 0.005)
    assert n[0] == times[2] and n[1] == times[6] and math.isinf(n[2])
    assert runner.steps_to_tolerance(times, np.repeat(Uinf[None], 8, axis=0), Uinf, 0.005)[0] == times[0]
