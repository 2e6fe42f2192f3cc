"""PD load balancing of the plane between two workers (Sec. 5.2, Eqs.
13-14): the oracle against hand-computed values and a closed loop whose
fixed point is known, then the library's host implementation against the
oracle.  Host-only code: no device is used."""
import math

import numpy as np
import pytest

from oracle.balance import PDBalance, imbalance
from paper_2605_15875_amd import abd


def test_imbalance_values():
    # eta = 3: T = (3 - 1) / (3 + 1); balanced: 0; swapped: the negative
    assert imbalance(3.0, 1.0) == pytest.approx(0.5, abs=1e-15)
    assert imbalance(1.0, 3.0) == pytest.approx(-0.5, abs=1e-15)
    assert imbalance(2.5, 2.5) == 0.0
    assert imbalance(9.0, 1.0) == pytest.approx(0.8, abs=1e-15)
    rng = np.random.default_rng(0)
    for a, b in rng.uniform(1e-3, 1e3, size=(200, 2)):
        t = imbalance(a, b)
        assert -1.0 < t < 1.0
        assert math.copysign(1.0, t) == math.copysign(1.0, a - b) or t == 0
        assert t == pytest.approx(-imbalance(b, a), abs=1e-15)


def test_pd_sequence_by_hand():
    c = PDBalance(k_p=-0.2, k_d=-0.1)
    # frame 1: T = 0.5, no derivative term yet: -0.2 * 0.5
    assert c.update(3.0, 1.0) == pytest.approx(-0.1, abs=1e-15)
    # frame 2: T = 0: -0.1 * (0 - 0.5)
    assert c.update(1.0, 1.0) == pytest.approx(0.05, abs=1e-15)
    # frame 3: T = -0.5: -0.2 * -0.5 + -0.1 * (-0.5 - 0)
    assert c.update(1.0, 3.0) == pytest.approx(0.15, abs=1e-15)


def test_smoothing_by_hand():
    c = PDBalance(k_p=1.0, k_d=10.0, smooth=0.5)
    assert c.update(2.0, 2.0) == 0.0            # tau = (2, 2), T = 0
    # tau = (0.5*2 + 0.5*4, 2) = (3, 2): eta 1.5, T = 0.5 / 2.5 = 0.2
    assert c.update(4.0, 2.0) == pytest.approx(0.2 + 10.0 * 0.2, abs=1e-14)
    # tau = (0.5*3 + 0.5*1, 0.5*2 + 0.5*2) = (2, 2): T = 0, dT = -0.2
    assert c.update(1.0, 2.0) == pytest.approx(-2.0, abs=1e-14)


def test_closed_loop_reaches_the_balanced_cut():
    """A plant where a worker's frame time is proportional to the number of
    bodies on its side of the cut (worker 1 below it): the balanced cut is
    the median of the body positions, and the controller with gains that
    shrink the slower side drives an uneven start there."""
    rng = np.random.default_rng(7)
    xs = np.sort(rng.gamma(2.0, 1.0, size=4000))   # skewed positions
    median = float(np.median(xs))
    span = float(xs[-1] - xs[0])
    cut = float(np.quantile(xs, 0.1))
    c = PDBalance(k_p=-0.3, k_d=-0.1, smooth=0.7)
    for _ in range(60):
        n1 = int(np.searchsorted(xs, cut))
        n1 = min(max(n1, 1), len(xs) - 1)
        cut += c.update(1e-3 * n1, 1e-3 * (len(xs) - n1)) * 1.0
    n1 = int(np.searchsorted(xs, cut))
    assert abs(cut - median) < 0.02 * span
    balance = (len(xs) / 2) / max(n1, len(xs) - n1)   # average / maximum
    assert balance > 0.97


def test_oracle_rejects_bad_input():
    with pytest.raises(ValueError):
        PDBalance(1.0, 0.0, smooth=0.0)
    with pytest.raises(ValueError):
        PDBalance(1.0, 0.0).update(0.0, 1.0)


def test_library_matches_oracle():
    rng = np.random.default_rng(3)
    for smooth in (1.0, 0.3):
        kp, kd = rng.uniform(-1.0, 1.0, size=2)
        ref = PDBalance(kp, kd, smooth)
        lib = abd.Balance(kp, kd, smooth)
        for t1, t2 in rng.uniform(1e-3, 5.0, size=(50, 2)):
            assert lib.update(t1, t2) == pytest.approx(
                ref.update(t1, t2), rel=1e-13, abs=1e-15)


def test_library_rejects_bad_input_and_keeps_state():
    b = abd.Balance(-0.2, -0.1)
    assert b.update(3.0, 1.0) == pytest.approx(-0.1)
    before = (tuple(b.st.tau), b.st.T_prev, b.st.frames)
    for t1, t2 in ((0.0, 1.0), (1.0, -2.0), (float("nan"), 1.0),
                   (1.0, float("inf"))):
        with pytest.raises(abd.AbdError):
            b.update(t1, t2)
    assert (tuple(b.st.tau), b.st.T_prev, b.st.frames) == before
    b.st.smooth = 1.5
    with pytest.raises(abd.AbdError):
        b.update(1.0, 1.0)
    b.st.smooth = 1.0
    # frame 2 as in the hand-computed sequence
    assert b.update(1.0, 1.0) == pytest.approx(0.05)
