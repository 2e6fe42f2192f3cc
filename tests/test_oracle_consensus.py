"""Pins of the consensus-side oracle (Eqs. 6, 7, 9, 10, 12, Sec. 4.2-4.3)
against independent facts: the Eq. 6 minimiser found by a generic
optimiser, hand-worked residuals, every branch and bound of the penalty
rule, and an ADMM run on quadratic local objectives whose monolithic
minimiser is known in closed form."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import consensus as K


def test_consensus_z_is_the_weighted_minimiser():
    rng = np.random.default_rng(0)
    group = np.array([0, 1, 0, 2, 1, 0])
    q = rng.normal(size=(6, 12))
    u = rng.normal(size=(6, 12)) * 0.1
    rho = rng.uniform(0.5, 5.0, 6)
    z = K.consensus_z(q, u, rho, group, 3)
    for b in range(3):
        idx = np.where(group == b)[0]

        def f(x):
            return sum(0.5 * rho[k] * np.sum((x - q[k] - u[k]) ** 2) for k in idx)

        res = minimize(f, np.zeros(12), method="BFGS", options=dict(gtol=1e-12))
        np.testing.assert_allclose(z[b], res.x, atol=1e-7)


def test_consensus_z_special_cases():
    q = np.arange(24, dtype=float).reshape(2, 12)
    u = np.ones((2, 12))
    # equal penalties: plain mean of q + u
    z = K.consensus_z(q, u, [3.0, 3.0], [0, 0], 1)
    np.testing.assert_array_equal(z[0], (q[0] + q[1]) / 2 + 1)
    # one replica: z = q + u exactly
    z1 = K.consensus_z(q[:1], u[:1], [7.0], [0], 1)
    np.testing.assert_array_equal(z1[0], q[0] + u[0])
    with pytest.raises(ValueError):
        K.consensus_z(q, u, [1.0, 1.0], [0, 0], 2)  # body 1 has no replica


def test_dual_update_and_residuals_by_hand():
    group = [0, 0, 1]
    q = np.zeros((3, 12))
    q[0, 0], q[1, 0], q[2, 5] = 1.0, 3.0, -2.0
    u = np.zeros((3, 12))
    z_old = np.zeros((2, 12))
    z = K.consensus_z(q, u, [1.0, 1.0, 1.0], group, 2)
    assert z[0, 0] == 2.0 and z[1, 5] == -2.0
    u2 = K.dual_update(u, q, z, group)
    assert u2[0, 0] == -1.0 and u2[1, 0] == 1.0 and np.all(u2[2] == 0)
    r_rep, s_body, r_inf, s_inf = K.residuals(q, z, z_old, group)
    np.testing.assert_array_equal(r_rep, [1.0, 1.0, 0.0])
    np.testing.assert_array_equal(s_body, [2.0, 2.0])
    assert r_inf == 1.0 and s_inf == 2.0
    # agreement: no residual, duals unchanged
    qa = np.ones((2, 12))
    za = K.consensus_z(qa, np.zeros((2, 12)), [1.0, 2.0], [0, 0], 1)
    np.testing.assert_array_equal(K.dual_update(np.zeros((2, 12)), qa, za, [0, 0]), 0)


def test_adapt_rho_branches_and_clamp():
    rho0 = np.array([10.0, 10.0, 10.0])
    u = np.ones((3, 12))
    group = [0, 1, 2]
    r_rep = np.array([6.0, 1.0, 1.0])
    s_body = np.array([1.0, 6.0, 1.0])
    rho, u2 = K.adapt_rho(rho0, rho0, u, r_rep, s_body, group)
    np.testing.assert_array_equal(rho, [20.0, 5.0, 10.0])
    # the unscaled dual rho * u is unchanged by the rescaling
    np.testing.assert_allclose(rho[:, None] * u2, rho0[:, None] * u)
    # the clamp: at sigma_max rho0 growth stops, at sigma_min shrink stops
    hi, _ = K.adapt_rho([1e4], [10.0], np.ones((1, 12)), [1.0], [0.0], [0])
    lo, _ = K.adapt_rho([1e-2], [10.0], np.ones((1, 12)), [0.0], [1.0], [0])
    assert hi[0] == 1e4 and lo[0] == 1e-2
    # replicas of one body share the body's largest residual
    rho, _ = K.adapt_rho([1.0, 1.0], [1.0, 1.0], np.zeros((2, 12)),
                         [0.0, 10.0], [1.0], [0, 0])
    np.testing.assert_array_equal(rho, [2.0, 2.0])


def test_mass_rho0_and_merge_target():
    np.testing.assert_array_equal(K.mass_rho0([2.0, 5.0], beta=0.5), [1.0, 2.5])
    qw = np.zeros((4, 12))
    m = K.merge_target(qw, [1, 3], np.ones((2, 12)))
    assert np.all(m[[1, 3]] == 1) and np.all(m[[0, 2]] == 0)
    assert np.all(qw == 0)


def test_admm_on_quadratics_reaches_the_monolithic_minimiser():
    """Workers i minimise 1/2 w_i |x - a_i|^2 over one shared body; the
    monolithic minimiser is sum w_i a_i / sum w_i.  Local solve (Eq. 5) in
    closed form, then Eqs. 6, 7 and the Eq. 12 penalty rule."""
    rng = np.random.default_rng(3)
    a = rng.normal(size=(3, 12))
    w = np.array([1.0, 4.0, 2.0])
    x_star = (w[:, None] * a).sum(0) / w.sum()
    group = [0, 0, 0]
    rho0 = np.full(3, 1.0)
    rho = rho0.copy()
    u = np.zeros((3, 12))
    z = a.mean(0, keepdims=True)
    for k in range(300):
        q = (w[:, None] * a + rho[:, None] * (z[0] - u)) / (w + rho)[:, None]
        z_new = K.consensus_z(q, u, rho, group, 1)
        u = K.dual_update(u, q, z_new, group)
        r_rep, s_body, r_inf, s_inf = K.residuals(q, z_new, z, group)
        z = z_new
        if r_inf < 1e-13 and s_inf < 1e-13:
            break
        rho, u = K.adapt_rho(rho, rho0, u, r_rep, s_body, group)
    np.testing.assert_allclose(z[0], x_star, atol=1e-11)


def test_oracle_admm_on_a_split_scene_reaches_the_monolithic_step():
    """Two subdomains of a row of four cubes in contact (gaps below d-hat),
    split at x = 0 with the two middle cubes shared: consensus ADMM with the
    oracle's local solves must end each time step where the monolithic
    solve of the whole scene ends."""
    from oracle import oracle as O
    from paper_2605_15875_amd import scenes
    th = 1e-8
    sc = scenes.cubes_scene(0, 4, 1, 1, gap=0.0006, jitter=0.0001,
                            newton_theta=th, pcg_eta=1e-12)
    sp = scenes.split_scene(sc, 0, 0.0, 1.2)
    assert sp.n_groups == 2 and len(sp.rep_prob) == 4
    mono = O.Oracle(sc)
    ws = [O.Oracle(w) for w in sp.workers]
    for w in ws:
        w.set_pair_replication(1)
    st = K.AdmmState(ws, sp, beta=1.0)
    for step in range(2):
        rep = K.admm_step(ws, st, sc.params["dt"], th, max_iters=300)
        assert rep["converged"] and rep["merge_ok"]
        so = mono.step()
        qm, qdm = mono.get_state()
        for w in range(2):
            qw, _ = ws[w].get_state()
            err = np.abs(qw - qm[sp.whole_ids[w]]).max() / so["scene_scale"]
            assert err < 1e-8, (step, w, err)
            ws[w].set_state(qm[sp.whole_ids[w]], qdm[sp.whole_ids[w]])
