"""List growth inside the device loop.  With every pair and candidate list
starting at a few entries, the first passes of a solve overflow them: the
overflow is detected on the device (the pass leaves the state as it was),
the host grows the lists, and the pass is run again with the full static
broad phase before later passes take lists over again.  Every time step
from the oracle's state must still land on the oracle's positions, for a
single context and for a batch of two."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

LISTS = ("n_body_pairs", "n_chunk_pairs", "n_cand_pt", "n_cand_ee",
         "n_cand_pg")


def contact_spheres(seed=3):
    return scenes.spheres_in_box_scene(
        seed, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45,
        r_lo=0.05, r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-7,
        pcg_eta=1e-12)


@pytest.mark.parametrize("cap", [16, 200])
def test_growth_in_device_loop_matches_oracle(cap):
    sc = contact_spheres()
    gpu = abd.Solver(sc, list_capacity=cap)
    ref = O.Oracle(sc)
    longest = 0
    for k in range(8):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        sg = gpu.step()
        so = ref.step()
        assert sg["status"] == so["status"] == 0, (cap, k)
        longest = max([longest] + [sg[n] for n in LISTS])
        err = np.abs(gpu.vertices() - ref.vertices()).max() / sg["scene_scale"]
        assert err < 1e-9, (cap, k, err)
    if cap == 16:
        assert longest > cap        # some list did grow
    gpu.close()


def test_growth_in_a_batch_matches_oracle():
    scs = [contact_spheres(3), contact_spheres(4)]
    refs = [O.Oracle(sc) for sc in scs]
    gpus = [abd.Solver(sc, list_capacity=16) for sc in scs]
    bt = abd.Batch(gpus)
    for step in range(4):
        for g, r in zip(gpus, refs):
            q, qd = r.get_state()
            g.set_state(q, qd)
            g.begin_step()
            r.begin_step()
        stats = bt.local_solve()
        for i, (g, r) in enumerate(zip(gpus, refs)):
            so = r.local_solve()
            assert stats[i]["status"] == so["status"] == 0, (step, i)
            l = stats[i]["scene_scale"]
            err = np.abs(g.vertices() - r.vertices()).max() / l
            assert err < 1e-9, (step, i, err)
            g.end_step()
            r.end_step()
    bt.close()
    for g in gpus:
        g.close()
