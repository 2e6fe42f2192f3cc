"""Mixed-precision form (Hessian blocks, PSD projection, assembly and the
PCG matvec in FP32; gradient, distances, CCD, energies and PCG dots in
FP64) against the FP64 oracle.  Each Newton iteration uses the FP64
gradient, so converged states match the FP64 solution to the Newton
tolerance; the FP32 Hessian only changes the path.  Errors are stated
against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu


def test_mixed_hessian_is_fp32_rounding_of_fp64():
    sc = scenes.config(0, newton_theta=1e-9, pcg_eta=1e-12)
    ref = O.Oracle(sc)
    for _ in range(15):
        ref.step()
    q, qd = ref.get_state()
    gpu = abd.Solver(sc, precision=1)
    gpu.set_state(q, qd)
    gpu.begin_step()
    ref.begin_step()
    eg, eo = gpu.eval(), ref.eval(q)
    # the gradient stays FP64
    assert np.abs(eg["g"] - eo["g"]).max() / np.abs(eo["g"]).max() < 1e-8
    # Hessian blocks: FP32 arithmetic (Jacobi and accumulation)
    s = np.abs(eo["Hdiag"]).max()
    err = np.abs(eg["Hdiag"] - eo["Hdiag"]).max() / s
    assert 0 < err < 1e-5
    gpu.close()


@pytest.mark.parametrize("theta", [1e-6, 1e-8])
def test_mixed_steps_match_fp64_oracle(theta):
    sc = scenes.config(0, newton_theta=theta, pcg_eta=1e-6)
    ref = O.Oracle(sc)
    gpu = abd.Solver(sc, precision=1)
    worst = 0.0
    for k in range(sc.steps):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        sg = gpu.step()
        ref.step()
        l = sg["scene_scale"]
        xg = gpu.vertices()
        err = np.abs(xg - ref.vertices()).max() / l
        worst = max(worst, err)
        # converged to the Newton tolerance on both sides
        assert err < 20 * theta * sc.params["dt"], (k, err)
        nc, md = ref.penetration(xg)
        assert nc == 0 and md > 0
    print(f"theta {theta}: worst position error / l = {worst:.2e}")
    gpu.close()


def test_mixed_spheres_converge_without_penetration():
    sc = scenes.spheres_in_box_scene(
        3, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45,
        r_lo=0.05, r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-6)
    ref = O.Oracle(sc)
    gpu = abd.Solver(sc, precision=1)
    for k in range(10):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        sg = gpu.step()
        ref.step()
        assert sg["status"] == 0
        xg = gpu.vertices()
        err = np.abs(xg - ref.vertices()).max() / sg["scene_scale"]
        assert err < 1e-6, (k, err)
        nc, md = ref.penetration(xg)
        assert nc == 0 and md > 0
    gpu.close()


def test_mixed_switch_to_fp64_continues_the_solve():
    """A mixed solve that is told to switch after two Newton iterations
    continues from its current iterate with FP64 Hessians: the switch and
    the FP32 share of the iterations are reported, no work is repeated, and
    the step lands on the oracle's step from the same state.  A solvable
    step with the default rule needs no switch, and the context is mixed
    again for its next solve."""
    sc = scenes.config(0, newton_theta=1e-9, pcg_eta=1e-12)
    ref = O.Oracle(sc, newton_theta=1e-9, pcg_eta=1e-12)
    for _ in range(10):  # contact starts at step 9
        ref.step()
    q, qd = ref.get_state()
    gpu = abd.Solver(sc, precision=1, mixed_switch=2)
    gpu.set_state(q, qd)
    st = gpu.step()
    sr = ref.step()
    assert st["status"] == 0
    assert st["fp64_fallback"] == 1
    assert 2 <= st["newton_fp32"] < st["newton_iters"], st
    err = np.abs(gpu.vertices() - ref.vertices()).max() / st["scene_scale"]
    assert err < 1e-9, err
    assert sr["newton_iters"] > 3
    # the default rule: no switch on a solvable step, all iterations FP32,
    # and the next solve starts in mixed precision again
    ok = abd.Solver(sc, precision=1)
    ok.set_state(q, qd)
    for _ in range(3):
        st = ok.step()
        assert st["status"] == 0 and st["fp64_fallback"] == 0
        assert st["newton_fp32"] == st["newton_iters"]
    gpu.set_state(q, qd)
    st = gpu.step()
    assert st["status"] == 0 and st["fp64_fallback"] == 1
    assert 2 <= st["newton_fp32"] < st["newton_iters"]
    gpu.close()
    ok.close()

