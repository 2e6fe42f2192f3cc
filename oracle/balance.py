"""Load balancing of the boundary plane between two workers, in plain
Python -- TEST INFRASTRUCTURE ONLY (imported by tests, never by the library
or its binding).

Sec. 5.2: a discrete-time PD controller moves the plane p_12 + s n_12 that
separates worker 1 from worker 2 (n_12 points from 1 to 2) from the
workers' smoothed per-frame compute times tau_1, tau_2:

* Eq. 13 -- eta = tau_1 / tau_2 and the normalised imbalance
            T = (eta - 1) / (eta + 1), in (-1, 1), 0 when balanced,
            positive when worker 1 is the slower one;
* Eq. 14 -- the shift dp = K_P T^k + K_D (T^k - T^{k-1}), applied as
            p_12 := p_12 + dp n_12.

Readings where the section is silent: the smoothing is an exponential
moving average tau^k = (1 - a) tau^{k-1} + a t^k started at the first
frame's times; the first frame has no derivative term (T^{-1} = T^0); the
formula is applied as printed, so with n_12 from worker 1 to worker 2 a
controller that shrinks the slower worker's side has negative gains.
"""
from __future__ import annotations


def imbalance(tau1, tau2):
    """Eq. 13 with eta = tau1 / tau2."""
    eta = tau1 / tau2
    return (eta - 1.0) / (eta + 1.0)


class PDBalance:
    """Eq. 14 over a sequence of frames, with smoothed times."""

    def __init__(self, k_p, k_d, smooth=1.0):
        if not (0.0 < smooth <= 1.0):
            raise ValueError("smooth must lie in (0, 1]")
        self.k_p, self.k_d, self.a = float(k_p), float(k_d), float(smooth)
        self.tau = None
        self.T_prev = None

    def update(self, t1, t2):
        """Times of the frame just finished -> shift of the plane along
        n_12."""
        if not (t1 > 0.0 and t2 > 0.0):
            raise ValueError("frame times must be positive")
        if self.tau is None:
            self.tau = [float(t1), float(t2)]
        else:
            self.tau = [(1.0 - self.a) * self.tau[0] + self.a * t1,
                        (1.0 - self.a) * self.tau[1] + self.a * t2]
        T = imbalance(self.tau[0], self.tau[1])
        Tp = T if self.T_prev is None else self.T_prev
        self.T_prev = T
        return self.k_p * T + self.k_d * (T - Tp)
