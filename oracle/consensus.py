"""Consensus side of the ADMM split in plain numpy, FP64 -- TEST
INFRASTRUCTURE ONLY (imported by tests and the smoke check, never by the
library or its binding).

Replicas: one row per (worker, shared body) copy.  `group[k]` is the shared
body of replica k; every group has at least one replica.  Arrays:
q, u [n_rep][12], rho [n_rep], z [n_groups][12].

* consensus_z   -- Eq. 6, the minimiser of sum_i rho_i/2 |z - (q_i + u_i)|^2
                   over the replicas of each body: the rho-weighted mean.
* dual_update   -- Eq. 7, u_i + q_i - z.
* residuals     -- Eq. 9 (r_i = q_i - z, inf-norm per replica and its max)
                   and Eq. 10 (s = z_new - z_old, inf-norm per body and max).
* adapt_rho     -- Eq. 12 per body with tau, mu and the clamp
                   [sigma_min rho0, sigma_max rho0]; the residual of body b
                   is the largest inf-norm over its replicas.  The scaled
                   duals are rescaled by rho_old / rho_new (the scaled-form
                   rule for a changed penalty; the paper does not state it).
* mass_rho0     -- mass-aware initial penalty rho0 = beta m_b (Sec. 4.3).
* merge_target  -- the merged state of Sec. 4.2: the worker's q with every
                   shared body replaced by its consensus z.
"""
from __future__ import annotations

import numpy as np


def consensus_z(q, u, rho, group, n_groups):
    """Eq. 6: z_b = sum_i rho_i (q_i + u_i) / sum_i rho_i over replicas i
    of body b."""
    q = np.asarray(q, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    num = np.zeros((n_groups, 12))
    den = np.zeros(n_groups)
    for k in range(len(group)):
        num[group[k]] += rho[k] * (q[k] + u[k])
        den[group[k]] += rho[k]
    if np.any(den <= 0):
        raise ValueError("every shared body needs a replica with rho > 0")
    return num / den[:, None]


def dual_update(u, q, z, group):
    """Eq. 7: u_i <- u_i + q_i - z_{b(i)}."""
    return np.asarray(u) + np.asarray(q) - np.asarray(z)[np.asarray(group)]


def residuals(q, z_new, z_old, group):
    """Eqs. 9-10: per-replica |q_i - z|_inf, per-body |z_new - z_old|_inf,
    and their maxima r_inf, s_inf."""
    r_rep = np.abs(np.asarray(q) - np.asarray(z_new)[np.asarray(group)]).max(axis=1)
    s_body = np.abs(np.asarray(z_new) - np.asarray(z_old)).max(axis=1)
    return r_rep, s_body, float(r_rep.max(initial=0.0)), float(s_body.max(initial=0.0))


def adapt_rho(rho, rho0, u, r_rep, s_body, group, tau=2.0, mu=5.0,
              sigma_min=1e-3, sigma_max=1e3):
    """Eq. 12 per body b: rho * tau if |r_b| > mu |s_b|, rho / tau if
    |s_b| > mu |r_b|, else unchanged; clamped to [sigma_min, sigma_max] x
    rho0.  |r_b| is the largest replica residual of b.  Every replica of b
    gets the new value; its scaled dual is multiplied by rho_old/rho_new."""
    rho = np.asarray(rho, dtype=np.float64).copy()
    u = np.asarray(u, dtype=np.float64).copy()
    group = np.asarray(group)
    n_groups = len(s_body)
    r_body = np.zeros(n_groups)
    for k in range(len(group)):
        r_body[group[k]] = max(r_body[group[k]], r_rep[k])
    for k in range(len(group)):
        b = group[k]
        new = rho[k]
        if r_body[b] > mu * s_body[b]:
            new = tau * rho[k]
        elif s_body[b] > mu * r_body[b]:
            new = rho[k] / tau
        new = min(max(new, sigma_min * rho0[k]), sigma_max * rho0[k])
        u[k] = u[k] * (rho[k] / new)
        rho[k] = new
    return rho, u


def mass_rho0(mass, beta=1.0):
    """Sec. 4.3: rho0 = beta m_b."""
    return beta * np.asarray(mass, dtype=np.float64)


def merge_target(q_worker, shared_ids, z_of_shared):
    """Sec. 4.2: the worker's state with every shared body replaced by z."""
    out = np.array(q_worker, dtype=np.float64, copy=True)
    out[np.asarray(shared_ids)] = z_of_shared
    return out


class AdmmState:
    """Penalties that persist across time steps (rho) and their starts."""

    def __init__(self, workers, split, beta=1.0, rho_fixed=0.0):
        self.split = split
        rho0 = np.zeros(len(split.rep_prob))
        for k in range(len(rho0)):
            M, _ = workers[split.rep_prob[k]].body_mass()
            m = M[split.rep_body[k], 0, 0]
            rho0[k] = mass_rho0(m, beta) if beta > 0 else rho_fixed
        self.rho0 = rho0
        self.rho = rho0.copy()
        cnt = np.bincount(split.rep_group, minlength=split.n_groups)
        self.kappa = cnt[split.rep_group].astype(np.int32)


def _push(workers, st, z, u):
    sp = st.split
    for w, wk in enumerate(workers):
        sel = np.nonzero(sp.rep_prob == w)[0]
        wk.set_shared(sp.rep_body[sel], z[sp.rep_group[sel]], u[sel],
                      st.rho[sel], st.kappa[sel])


def _replica_q(workers, sp):
    qs = [wk.get_state()[0] for wk in workers]
    return np.array([qs[sp.rep_prob[k]][sp.rep_body[k]]
                     for k in range(len(sp.rep_prob))]), qs


def admm_step(workers, st, dt, theta, tau=2.0, mu=5.0, sigma_min=1e-3,
              sigma_max=1e3, scale=0.0, adapt=True, merge_check=True,
              max_iters=50):
    """One time step of consensus ADMM over the workers (Alg. 1): z = q~,
    u = 0; local solve (Eq. 5); then per round: Eqs. 6-7, the stopping
    tests of Eq. 8 with Eqs. 9-10, the merge check of Sec. 4.2 (ACCD of
    each worker toward its merged state must give TOI = 1), Eq. 12, and
    the next local solve.  On success every replica takes z."""
    sp = st.split
    for wk in workers:
        wk.begin_step()
    qt_rep = np.array([workers[sp.rep_prob[k]].qtilde()[sp.rep_body[k]]
                       for k in range(len(sp.rep_prob))])
    z = consensus_z(qt_rep, np.zeros_like(qt_rep), st.rho, sp.rep_group,
                    sp.n_groups)
    u = np.zeros((len(sp.rep_prob), 12))
    _push(workers, st, z, u)
    rep = dict(iters=0, converged=False, merge_ok=False, newton_iters_total=0)
    stats = None

    def update():
        nonlocal z, u
        q_rep, qs = _replica_q(workers, sp)
        z_new = consensus_z(q_rep, u, st.rho, sp.rep_group, sp.n_groups)
        u = dual_update(u, q_rep, z_new, sp.rep_group)
        r_rep, s_body, r_inf, s_inf = residuals(q_rep, z_new, z, sp.rep_group)
        z = z_new
        min_toi = 1.0
        if merge_check:
            for w, wk in enumerate(workers):
                sel = np.nonzero(sp.rep_prob == w)[0]
                target = merge_target(qs[w], sp.rep_body[sel], z[sp.rep_group[sel]])
                min_toi = min(min_toi, min(1.0, wk.ccd(qs[w], target - qs[w])))
        l = scale if scale > 0 else max(s_["scene_scale"] for s_ in stats)
        eps = max(s_["final_eps_N"] for s_ in stats)
        rep.update(eps_newton=eps, r_inf=r_inf / (dt * l), s_inf=s_inf / (dt * l),
                   min_toi=min_toi, merge_ok=min_toi >= 1.0)
        rep["converged"] = (eps < theta and rep["r_inf"] < theta and
                            rep["s_inf"] < theta and
                            (not merge_check or rep["merge_ok"]))
        return r_rep, s_body

    for k in range(1, max_iters + 1):
        if k > 1:
            r_rep, s_body = update()
            if rep["converged"]:
                break
            if adapt:
                st.rho, u = adapt_rho(st.rho, st.rho0, u, r_rep, s_body,
                                      sp.rep_group, tau, mu, sigma_min, sigma_max)
            _push(workers, st, z, u)
        stats = [wk.local_solve() for wk in workers]
        rep["iters"] = k
        rep["newton_iters_total"] += sum(s_["newton_iters"] for s_ in stats)
        if k == max_iters:
            update()
    if rep["converged"] or rep["merge_ok"]:
        q_rep, qs = _replica_q(workers, sp)
        for w, wk in enumerate(workers):
            sel = np.nonzero(sp.rep_prob == w)[0]
            wk.set_state(merge_target(qs[w], sp.rep_body[sel], z[sp.rep_group[sel]]))
    for wk in workers:
        wk.end_step()
    return rep
