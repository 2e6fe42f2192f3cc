"""The allocation-free solve (abd_local_solve_static) against the
allocating one (abd_local_solve) through the C-ABI: two calls in a row on
one GPU, the second on a smaller scene, each compared with a twin context
solved the ordinary way from the same state; both land on the same step
(positions within 1e-9 of the scene scale, the bar of the oracle parity,
at theta = 1e-9 on the cubes and 1e-7 on the contact-rich spheres, whose
last Newton steps at tighter tolerances sit at the rounding floor of the
barrier energy sum), and the static solve takes nothing from a bound
workspace, so it allocates no buffer of the context."""
import numpy as np
import pytest
import torch

from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

PARITY = dict(newton_theta=1e-9, pcg_eta=1e-12)
PARITY_CONTACT = dict(newton_theta=1e-7, pcg_eta=1e-12)


def _spheres():
    return scenes.spheres_in_box_scene(
        3, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45, r_lo=0.05,
        r_hi=0.08, min_gap=0.0005, vel=0.5, **PARITY_CONTACT)


def _advance(sc, steps):
    """A state with contacts: `steps` ordinary time steps."""
    s = abd.Solver(sc)
    for _ in range(steps):
        s.step()
    q, qd = s.get_state()
    s.close()
    return q, qd


def _one_step(sol, static):
    sol.begin_step()
    st = sol.local_solve_static() if static else sol.local_solve()
    sol.end_step()
    return st


def _compare(sc, q, qd, ws_bytes):
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    a = abd.Solver(sc, workspace=ws)  # the allocation-free solve
    b = abd.Solver(sc)                # the ordinary one
    for s in (a, b):
        s.set_state(q, qd)
    before = a.workspace_info()
    sa = _one_step(a, True)
    sb = _one_step(b, False)
    after = a.workspace_info()
    assert sa["status"] == 0 and sb["status"] == 0
    assert sa["n_active"] > 0  # the step has contacts
    assert after == before  # no buffer taken from the workspace
    l = sb["scene_scale"]
    err = np.abs(a.vertices() - b.vertices()).max() / l
    assert err < 1e-9, err
    qa, qda = a.get_state()
    qb, qdb = b.get_state()
    assert np.abs(qda - qdb).max() * sc.params["dt"] < 1e-9 * l
    a.close()
    b.close()
    return sa


def test_static_solve_matches_the_allocating_solve_twice_in_a_row():
    torch.cuda.set_device(0)
    big = _spheres()
    small = scenes.config(0, **PARITY)
    qb, qdb = _advance(big, 6)
    qs, qds = _advance(small, 10)
    s1 = _compare(big, qb, qdb, 64 << 20)
    s2 = _compare(small, qs, qds, 16 << 20)  # second call, smaller input
    assert s2["n_cand_pt"] + s2["n_cand_ee"] < s1["n_cand_pt"] + s1["n_cand_ee"]


def test_static_solve_in_mixed_precision_and_after_ordinary_solves():
    """The context keeps working both ways: ordinary, static, ordinary.
    Mixed precision at theta = 1e-6, the tolerance of the other mixed
    tests on these spheres: at tighter tolerances a step of the contact pile
    can need hundreds of Newton iterations in either precision (a small
    sphere turning on a vertex of its mesh, whose negative curvature the
    PSD projection clamps)."""
    torch.cuda.set_device(0)
    sc = scenes.spheres_in_box_scene(
        3, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45, r_lo=0.05,
        r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-6)
    q, qd = _advance(sc, 6)
    a = abd.Solver(sc, precision=1)
    b = abd.Solver(sc, precision=1)
    for s in (a, b):
        s.set_state(q, qd)
    for static in (False, True, False):
        sa = _one_step(a, static)
        sb = _one_step(b, False)
        assert sa["status"] == 0 and sb["status"] == 0
        err = np.abs(a.vertices() - b.vertices()).max() / sb["scene_scale"]
        assert err < 1e-6, (static, err)
        qq, qqd = b.get_state()
        a.set_state(qq, qqd)
    a.close()
    b.close()
