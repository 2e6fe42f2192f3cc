"""Device consensus ADMM over two subdomains solved as one batch: the
z/u/rho updates against the numpy oracle on the same replica states, whole
ADMM time steps against the oracle's ADMM and against the monolithic solve,
and the merge check of Sec. 4.2 on a merge that a static wall blocks."""
import numpy as np
import pytest

from oracle import consensus as K
from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

TH = 1e-8


def split_cubes(nx=4, ny=1):
    sc = scenes.cubes_scene(0, nx, ny, 1, gap=0.0006, jitter=0.0001,
                            newton_theta=TH, pcg_eta=1e-12)
    return sc, scenes.split_scene(sc, 0, 0.0, 1.2)


def device_admm(sp, **kw):
    gs = [abd.Solver(w) for w in sp.workers]
    for g in gs:
        g.set_pair_replication(1)
    bt = abd.Batch(gs)
    cs = abd.Consensus(bt, sp.rep_prob, sp.rep_body, sp.rep_group,
                       sp.n_groups, **kw)
    return gs, bt, cs


def test_consensus_updates_match_numpy_on_device_states():
    sc, sp = split_cubes(4, 2)
    gs, bt, cs = device_admm(sp, max_iters=50)
    for g in gs:
        g.begin_step()
    cs.begin()
    z0, u0, rho0 = cs.get()
    qt = np.array([gs[p].qtilde()[b] for p, b in zip(sp.rep_prob, sp.rep_body)])
    np.testing.assert_allclose(z0, K.consensus_z(qt, 0 * qt, rho0, sp.rep_group,
                                                 sp.n_groups), rtol=1e-15, atol=0)
    assert np.all(u0 == 0)
    # mass-aware start: rho0 = m_b (unit cubes of density 1000)
    np.testing.assert_allclose(rho0, 1000.0, rtol=1e-12)
    z, u, rho = z0, u0, rho0
    for k in range(4):
        bt.local_solve()
        q = np.array([gs[p].get_state()[0][b] for p, b in zip(sp.rep_prob, sp.rep_body)])
        rep = cs.update()
        z_ref = K.consensus_z(q, u, rho, sp.rep_group, sp.n_groups)
        u_ref = K.dual_update(u, q, z_ref, sp.rep_group)
        r_rep, s_body, r_inf, s_inf = K.residuals(q, z_ref, z, sp.rep_group)
        z_d, u_d, _ = cs.get()
        np.testing.assert_allclose(z_d, z_ref, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(u_d, u_ref, rtol=1e-12, atol=1e-15)
        assert rep["r_inf"] * sc.params["dt"] > 0.0 or r_inf == 0.0
        cs.adapt()
        rho_ref, u_ref2 = K.adapt_rho(rho, rho0, u_ref, r_rep, s_body, sp.rep_group)
        _, u_d2, rho_d = cs.get()
        np.testing.assert_array_equal(rho_d, rho_ref)
        np.testing.assert_allclose(u_d2, u_ref2, rtol=1e-12, atol=1e-15)
        z, u, rho = z_d, u_d2, rho_d
    cs.close()


def test_admm_steps_match_oracle_admm_and_monolithic():
    sc, sp = split_cubes(4, 1)
    gs, bt, cs = device_admm(sp, max_iters=300)
    ws = [O.Oracle(w) for w in sp.workers]
    for w in ws:
        w.set_pair_replication(1)
    st = K.AdmmState(ws, sp, beta=1.0)
    mono = O.Oracle(sc)
    for step in range(2):
        rg = cs.admm_step()
        ro = K.admm_step(ws, st, sc.params["dt"], TH, max_iters=300)
        so = mono.step()
        assert rg["converged"] and ro["converged"] and rg["merge_ok"]
        l = so["scene_scale"]
        qm, qdm = mono.get_state()
        for w in range(2):
            qg, _ = gs[w].get_state()
            qo, _ = ws[w].get_state()
            assert np.abs(qg - qo).max() / l < 1e-9, (step, w)
            assert np.abs(qg - qm[sp.whole_ids[w]]).max() / l < 1e-8, (step, w)
            # both continue from the monolithic state
            gs[w].set_state(qm[sp.whole_ids[w]], qdm[sp.whole_ids[w]])
            ws[w].set_state(qm[sp.whole_ids[w]], qdm[sp.whole_ids[w]])
    cs.close()


def blocked_split():
    """One shared cube; worker 1's copy starts with a large +x velocity and
    moves through free space, worker 0's copy sees a static wall in its
    path, so the consensus z lies beyond the wall for worker 0."""
    v, t = scenes.cube_mesh(0.5)
    wv, wt = scenes.cube_mesh(0.5)
    wv = wv * np.array([0.1, 4.0, 4.0])
    p = dict(scenes.default_params(has_ground=0, gravity=(0.0, 0.0, 0.0)),
             newton_theta=1e-6)
    cube0 = scenes.Body(v, t, 1000.0, scenes.identity_q([0, 0, 0]),
                        np.zeros(12), scenes.DYNAMIC)
    wall = scenes.Body(wv, wt, 1000.0, scenes.identity_q([0.7, 0, 0]),
                       np.zeros(12), scenes.STATIC)
    qd = np.zeros(12)
    qd[0] = 150.0
    cube1 = scenes.Body(v, t, 1000.0, scenes.identity_q([0, 0, 0]), qd,
                        scenes.DYNAMIC)
    w0 = scenes.Scene("w0", p, [cube0, wall], 1)
    w1 = scenes.Scene("w1", dict(p), [cube1], 1)
    return scenes.Split([w0, w1], np.array([0, 1], dtype=np.int32),
                        np.array([0, 0], dtype=np.int32),
                        np.array([0, 0], dtype=np.int32), 1,
                        [np.array([0, 1]), np.array([0])])


def test_merge_check_reports_a_blocked_merge():
    sp = blocked_split()
    gs, bt, cs = device_admm(sp, max_iters=50)
    ws = [O.Oracle(w) for w in sp.workers]
    for w in ws:
        w.set_pair_replication(1)
    for g in gs:
        g.begin_step()
    cs.begin()
    bt.local_solve()
    rep = cs.update()
    assert not rep["merge_ok"] and rep["min_toi"] < 1.0
    assert not rep["converged"]
    # the oracle's merge check on the same states agrees
    z, _, _ = cs.get()
    q0, _ = gs[0].get_state()
    tgt = K.merge_target(q0, [0], z)
    ws[0].set_state(q0)
    assert ws[0].ccd(q0, tgt - q0) < 1.0
    cs.close()
