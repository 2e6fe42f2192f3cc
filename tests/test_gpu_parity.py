"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Tolerances: candidate sets bit-exact after sorting (exact predicate on the
library's exported positions); gradients and Hessian blocks 1e-8 relative
to the largest entry; positions 1e-9 of the scene scale after a step from
a shared start state; the GPU's CCD step never above the oracle's.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

PARITY = dict(newton_theta=1e-9, pcg_eta=1e-12)
# contact-rich scenes: at theta 1e-9 the last Newton steps fall below the
# rounding of the barrier energy sum on both sides (the oracle itself stops
# with NOCONV), so they are compared at 1e-8
PARITY_CONTACT = dict(newton_theta=1e-8, pcg_eta=1e-12)


def rel(a, b):
    s = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / s)


@pytest.fixture(scope="module")
def cubes_contact():
    """8-cube scene advanced by the oracle into resting + stacking contact."""
    sc = scenes.config(0, **PARITY)
    ref = O.Oracle(sc)
    states = []
    for _ in range(16):
        states.append(ref.get_state())
        ref.step()
    return sc, ref, states


@pytest.fixture(scope="module")
def cubes_gpu(cubes_contact):
    sc, _, _ = cubes_contact
    s = abd.Solver(sc)
    yield s
    s.close()


def set_both(gpu, ref, q, qd):
    gpu.set_state(q, qd)
    ref.set_state(q, qd)
    gpu.begin_step()
    ref.begin_step()


def test_prediction_and_positions(cubes_contact, cubes_gpu):
    sc, ref, states = cubes_contact
    q, qd = states[14]
    set_both(cubes_gpu, ref, q, qd)
    assert rel(cubes_gpu.qtilde(), ref.qtilde()) < 1e-15
    np.testing.assert_allclose(cubes_gpu.vertices(), ref.vertices(),
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [10, 13, 15])
def test_candidates_bitexact(cubes_contact, cubes_gpu, k):
    sc, ref, states = cubes_contact
    q, qd = states[k]
    set_both(cubes_gpu, ref, q, qd)
    x = cubes_gpu.vertices()
    for kind in (O.PT, O.EE, O.PG):
        np.testing.assert_array_equal(cubes_gpu.candidates(kind),
                                      ref.candidates(kind, x))
    dq, _ = ref.direction(q)
    x2, dx = cubes_gpu.vertices(None, dq)
    for kind in (O.PT, O.EE, O.PG):
        np.testing.assert_array_equal(cubes_gpu.candidates(kind, dq),
                                      ref.candidates(kind, x2, dx))


@pytest.mark.parametrize("k", [10, 13, 15])
def test_eval_parity(cubes_contact, cubes_gpu, k):
    sc, ref, states = cubes_contact
    q, qd = states[k]
    set_both(cubes_gpu, ref, q, qd)
    eg, eo = cubes_gpu.eval(), ref.eval(q)
    assert eg["n_active"] == eo["n_active"] > 0
    assert eg["E"] == pytest.approx(eo["E"], rel=1e-12)
    assert rel(eg["g"], eo["g"]) < 1e-8
    assert rel(eg["Hdiag"], eo["Hdiag"]) < 1e-8
    np.testing.assert_array_equal(eg["off_ij"], eo["off_ij"])
    if len(eo["off_ij"]):
        assert rel(eg["Hoff"], eo["Hoff"]) < 1e-8


def test_direction_ccd_energy_parity(cubes_contact, cubes_gpu):
    sc, ref, states = cubes_contact
    for k in (9, 13, 15):
        q, qd = states[k]
        set_both(cubes_gpu, ref, q, qd)
        dq_o, _ = ref.direction(q)
        dq_g, it = cubes_gpu.direction()
        assert rel(dq_g, dq_o) < 1e-8
        ag, ao = cubes_gpu.ccd(dq_o), ref.ccd(q, dq_o)
        assert ag <= ao * (1 + 1e-12)
        assert ag == pytest.approx(ao, rel=1e-9)
        for a in (ao, 0.5 * ao):
            dg = cubes_gpu.energy_delta(dq_o, a)
            do = ref.energy_delta(q, dq_o, a)
            assert dg == pytest.approx(do, rel=1e-7, abs=1e-14)


def test_per_pair_toi_parity(cubes_contact, cubes_gpu):
    """Each swept candidate's own time of impact against the oracle's
    additive CCD of that pair (positions and step from the oracle's vertex
    map), in the exported candidate order, and alpha_max as their
    minimum."""
    sc, ref, states = cubes_contact
    offs = np.cumsum([0] + [len(b.xbar) for b in sc.bodies[:-1]])
    tris = np.concatenate([b.tris + o for b, o in zip(sc.bodies, offs)])
    edges = ref.edges()
    s = 0.1                      # additive-CCD gap fraction of both sides
    impacts = 0
    for k in (9, 13, 15):
        q, qd = states[k]
        set_both(cubes_gpu, ref, q, qd)
        dq, _ = ref.direction(q)
        for scale in (1.0, 4.0):       # a longer step reaches more contacts
            d = scale * dq
            a, toi = cubes_gpu.ccd(d, per_pair=True)
            pt, ee, pg = (cubes_gpu.candidates(kd, d)
                          for kd in (O.PT, O.EE, O.PG))
            assert len(toi) == len(pt) + len(ee) + len(pg) > 0
            x, dx = ref.vertices(q), ref.vertices(d)   # dx = J d (linear)
            want, exact = [], []
            for kd, pairs in ((O.PT, pt), (O.EE, ee)):
                for i, j in pairs:
                    vid = ([i, *tris[j]] if kd == O.PT
                           else [*edges[i], *edges[j]])
                    want.append(O.accd(kd, x[vid].ravel(), dx[vid].ravel(),
                                       s))
                    exact.append(O.exact_toi(kd, x[vid].ravel(),
                                             dx[vid].ravel()))
            for v in pg:
                dy = dx[v, 1]
                y0 = x[v, 1] - sc.params["ground_y"]
                want.append((1 - s) * y0 / -dy if dy < 0 else 1.0)
                exact.append(min(1.0, y0 / -dy) if dy < 0 else 1.0)
            want = np.clip(np.array(want), 0.0, 1.0)
            np.testing.assert_allclose(toi, want, rtol=1e-9, atol=1e-15)
            # the CCD contract: never beyond the exact first contact
            assert np.all(toi <= np.array(exact)), "TOI above exact contact"
            assert a == min(1.0, float(toi.min()))
            impacts += int((toi < 1.0).sum())
    assert impacts > 0


def test_step_parity_from_shared_state(cubes_contact, cubes_gpu):
    """Each time step of the 8-cube run from the oracle's start state:
    positions within 1e-9 of the scene scale, same Newton iteration
    count, no penetration."""
    sc, ref0, states = cubes_contact
    ref = O.Oracle(sc)
    for k in range(16):
        q, qd = states[k]
        cubes_gpu.set_state(q, qd)
        ref.set_state(q, qd)
        sg = cubes_gpu.step()
        so = ref.step()
        l = sg["scene_scale"]
        assert l == pytest.approx(so["scene_scale"], rel=1e-14)
        err = np.abs(cubes_gpu.vertices() - ref.vertices()).max() / l
        assert err < 1e-9, (k, err)
        assert sg["newton_iters"] == so["newton_iters"]
        nc, md = ref.penetration(cubes_gpu.vertices())
        assert nc == 0 and md > 0


def test_free_running_cubes_stay_close_and_feasible():
    sc = scenes.config(0, **PARITY)
    gpu = abd.Solver(sc)
    ref = O.Oracle(sc)
    for k in range(sc.steps):
        gpu.step()
        ref.step()
        xg = gpu.vertices()
        l = np.linalg.norm(np.ptp(xg, axis=0))
        assert np.abs(xg - ref.vertices()).max() / l < 1e-7 * (k + 1)
        nc, md = ref.penetration(xg)
        assert nc == 0 and md > 0
    gpu.close()


def test_free_fall_closed_form_gpu():
    v_, t_ = scenes.cube_mesh(0.5)
    qd = np.zeros(12)
    qd[:3] = [0.3, 0.7, -0.2]
    sc = scenes.Scene("cube", scenes.default_params(newton_theta=1e-10),
                      [scenes.Body(v_, t_, 1000.0,
                                   scenes.identity_q([0, 5, 0]), qd)], 1)
    gpu = abd.Solver(sc)
    h, g = sc.params["dt"], np.array(sc.params["gravity"])
    for n in range(1, 11):
        gpu.step()
        q, _ = gpu.get_state()
        ref = np.array([0, 5, 0]) + n * h * qd[:3] + h * h * g * n * (n + 1) / 2
        np.testing.assert_allclose(q[0, :3], ref, atol=1e-12)
    gpu.close()


def small_spheres(seed=3):
    # theta 1e-7: at 1e-8 the last Newton steps of this contact-rich scene
    # sit at the rounding floor of the energy sum, where the line search
    # halves at random and the order of the device's floating-point
    # accumulations (which varies run to run) decides how many iterations
    # are needed
    return scenes.spheres_in_box_scene(
        seed, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45,
        r_lo=0.05, r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-7,
        pcg_eta=1e-12)


def test_spheres_in_box_parity():
    """Spheres (with a static container: PT/EE against large static
    triangles, off-diagonal blocks between dynamic bodies) stepped from
    shared states."""
    sc = small_spheres()
    gpu = abd.Solver(sc)
    ref = O.Oracle(sc)
    saw_contact = False
    for k in range(12):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        gpu.begin_step()
        ref.begin_step()
        x = gpu.vertices()
        for kind in (O.PT, O.EE):
            np.testing.assert_array_equal(gpu.candidates(kind),
                                          ref.candidates(kind, x))
        eg, eo = gpu.eval(), ref.eval(q)
        assert rel(eg["g"], eo["g"]) < 1e-8
        assert rel(eg["Hdiag"], eo["Hdiag"]) < 1e-8
        np.testing.assert_array_equal(eg["off_ij"], eo["off_ij"])
        saw_contact |= eo["n_active"] > 0
        gpu.set_state(q, qd)
        sg = gpu.step()
        ref.step()
        l = sg["scene_scale"]
        assert np.abs(gpu.vertices() - ref.vertices()).max() / l < 1e-9
    assert saw_contact
    gpu.close()


def test_admm_penalty_and_replication_parity(cubes_contact):
    """Shared bodies with z, u, rho and kappa_b = 2, and the by-shared-set
    pair replication rule: gradient, Hessian and one local solve match."""
    sc, ref0, states = cubes_contact
    q, qd = states[15]
    rng = np.random.default_rng(7)
    ids = np.array([0, 2, 4, 6], dtype=np.int32)
    gpu = abd.Solver(sc)
    ref = O.Oracle(sc)
    for s in (gpu, ref):
        s.set_state(q, qd)
        s.begin_step()
    qt = ref.qtilde()
    z = qt[ids] + np.concatenate([rng.uniform(-1e-3, 1e-3, (4, 3)),
                                  rng.uniform(-1e-4, 1e-4, (4, 9))], axis=1)
    u = rng.uniform(-1e-5, 1e-5, (4, 12))
    rho = np.full(4, 1e4)
    kb = np.full(4, 2, np.int32)
    for s in (gpu, ref):
        s.set_shared(ids, z, u, rho, kb)
        s.set_pair_replication(1)
    eg, eo = gpu.eval(), ref.eval(q)
    assert eg["E"] == pytest.approx(eo["E"], rel=1e-12)
    assert rel(eg["g"], eo["g"]) < 1e-8
    assert rel(eg["Hdiag"], eo["Hdiag"]) < 1e-8
    sg = gpu.local_solve()
    so = ref.local_solve()
    assert sg["newton_iters"] == so["newton_iters"]
    l = sg["scene_scale"]
    assert np.abs(gpu.vertices() - ref.vertices()).max() / l < 1e-9
    gpu.close()


def test_error_paths():
    v, t = scenes.cube_mesh(0.5)
    # the second cube's bottom vertices lie exactly on the first's top face
    overlap = scenes.Scene("touch", scenes.default_params(), [
        scenes.Body(v, t, 1000.0, scenes.identity_q([0, 2, 0]), np.zeros(12)),
        scenes.Body(v, t, 1000.0, scenes.identity_q([0.25, 3.0, 0.125]),
                    np.zeros(12))], 1)
    with pytest.raises(abd.AbdError) as e:
        abd.Solver(overlap)
    assert e.value.code == abd.E_INFEASIBLE
    # interpenetrating cubes whose closest features are all > 0 apart: the
    # edge-triangle crossing check rejects them
    deep = scenes.Scene("deep", scenes.default_params(), [
        scenes.Body(v, t, 1000.0, scenes.identity_q([0, 2, 0]), np.zeros(12)),
        scenes.Body(v, t, 1000.0, scenes.identity_q([0.5, 2.3, 0.1]),
                    np.zeros(12))], 1)
    with pytest.raises(abd.AbdError) as e:
        abd.Solver(deep)
    assert e.value.code == abd.E_INFEASIBLE
    sc = scenes.config(0)
    gpu = abd.Solver(sc)
    with pytest.raises(abd.AbdError) as e:
        z = np.zeros((1, 12))
        z[0, 3] = np.nan
        gpu.set_shared([0], z, np.zeros((1, 12)), [1e4], [2])
    assert e.value.code == abd.E_INVALID_ARG
    gpu.close()
    # max_newton = 1 in a step that needs more: NOCONV, state = last iterate
    sc = scenes.config(0, max_newton=1)
    gpu = abd.Solver(sc)
    gpu.begin_step()
    st = gpu.local_solve(check=False)
    assert st["status"] == abd.E_NOCONV and st["newton_iters"] == 1
    q, _ = gpu.get_state()
    assert np.all(np.isfinite(q))
    gpu.close()


def test_spheres_toi_never_above_exact_contact():
    """Sphere scene (PT/EE between curved meshes and against the static
    box): every swept pair's GPU time of impact stays at or below the
    oracle's exact first contact time of that pair, for the Newton step and
    for steps stretched until many pairs would collide."""
    sc = small_spheres()
    gpu = abd.Solver(sc)
    ref = O.Oracle(sc)
    offs = np.cumsum([0] + [len(b.xbar) for b in sc.bodies[:-1]])
    tris = np.concatenate([b.tris + o for b, o in zip(sc.bodies, offs)])
    edges = ref.edges()
    impacts = 0
    for k in range(10):
        q, qd = ref.get_state()
        if k in (4, 7, 9):
            set_both(gpu, ref, q, qd)
            dq, _ = ref.direction(q)
            for scale in (1.0, 8.0, 40.0):
                d = scale * dq
                a, toi = gpu.ccd(d, per_pair=True)
                pt, ee, pg = (gpu.candidates(kd, d) for kd in (O.PT, O.EE, O.PG))
                x, dx = ref.vertices(q), ref.vertices(d)
                exact = []
                for kd, pairs in ((O.PT, pt), (O.EE, ee)):
                    for i, j in pairs:
                        vid = ([i, *tris[j]] if kd == O.PT
                               else [*edges[i], *edges[j]])
                        exact.append(O.exact_toi(kd, x[vid].ravel(),
                                                 dx[vid].ravel()))
                assert len(pg) == 0
                exact = np.array(exact)
                assert len(toi) == len(exact)
                assert np.all(toi <= exact), (k, scale)
                assert a <= exact.min(initial=1.0)
                impacts += int((exact < 1.0).sum())
        ref.step()
    assert impacts > 0
    gpu.close()


def test_cooperative_launch_setting_is_rejected(cubes_gpu):
    with pytest.raises(abd.AbdError) as e:
        cubes_gpu.set_tuning(pcg_coop=1)
    assert e.value.code == abd.E_INVALID_ARG
