"""Context buffers in caller-owned device memory (a PyTorch tensor): solves
from the oracle's state land on the oracle's positions, lists grown inside
the device loop take their space from the workspace, and a workspace that
is too small, bound late or not device memory is refused with an error."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu


def contact_spheres():
    return scenes.spheres_in_box_scene(
        3, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45,
        r_lo=0.05, r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-7,
        pcg_eta=1e-12)


def test_workspace_solves_match_oracle_and_hold_the_growth():
    sc = contact_spheres()
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    gpu = abd.Solver(sc, workspace=ws, list_capacity=16)
    size, used0, _ = gpu.workspace_info()
    assert 0 < used0 <= size <= ws.numel()
    ref = O.Oracle(sc)
    for k in range(6):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        sg = gpu.step()
        so = ref.step()
        assert sg["status"] == so["status"] == 0, k
        err = np.abs(gpu.vertices() - ref.vertices()).max() / sg["scene_scale"]
        assert err < 1e-9, (k, err)
    size, used, peak = gpu.workspace_info()
    assert used > used0 and used <= peak <= size   # grown lists came from it
    # the state lives in the tensor: clearing the tensor clears it
    ws.zero_()
    torch.cuda.synchronize()
    q, qd = gpu.get_state()
    assert not q.any() and not qd.any()
    gpu.close()
    del ws


def test_workspace_matches_library_memory_on_cubes():
    sc = scenes.cubes_scene(0, 2, 2, 2)
    ws = torch.empty(16 << 20, dtype=torch.uint8, device="cuda:0")
    a = abd.Solver(sc, workspace=ws)
    b = abd.Solver(sc)
    for k in range(10):
        sa, sb = a.step(), b.step()
        assert sa["status"] == sb["status"] == 0
        l = sa["scene_scale"]
        # same kernels; only the order of floating-point atomics may differ
        assert np.abs(a.vertices() - b.vertices()).max() / l < 1e-9, k
    assert b.workspace_info() == (0, 0, 0)
    a.close()
    b.close()


def test_small_workspace_fails_cleanly_and_the_device_stays_usable():
    sc = contact_spheres()
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(abd.AbdError) as e:
        abd.Solver(sc, workspace=ws)
    assert e.value.code == abd.E_OOM and "workspace" in str(e.value)
    s = abd.Solver(scenes.cubes_scene(0, 2, 2, 2))
    assert s.step()["status"] == 0
    s.close()


def test_bind_is_refused_late_twice_or_on_host_memory():
    sc = scenes.cubes_scene(0, 2, 2, 2)
    L = abd.lib()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    s = abd.Solver(sc)                       # finalized: too late
    assert L.abd_bind_workspace(s.h, ws.data_ptr(), ws.numel()) == \
        abd.E_INVALID_ARG
    s.close()
    s = abd.Solver(sc, finalize=False)
    host = np.zeros(1 << 16, dtype=np.uint8)
    assert L.abd_bind_workspace(s.h, host.ctypes.data, host.nbytes) == \
        abd.E_INVALID_ARG
    assert L.abd_bind_workspace(s.h, ws.data_ptr(), 100) == abd.E_INVALID_ARG
    assert L.abd_bind_workspace(s.h, ws.data_ptr(), ws.numel()) == abd.OK
    assert L.abd_bind_workspace(s.h, ws.data_ptr(), ws.numel()) == \
        abd.E_INVALID_ARG                    # bound once
    s.close()
