"""The device loop's launch paths give the same solve: whole passes replayed
from one captured graph (no timing), passes in two captured halves around
an event-timed PCG launch (every fourth pass with PCG timing), direct
launches with every stage timed, and direct launches (the default) with
and without PCG timing.  From the oracle's state
each time step lands on the oracle's positions, and the timed modes report
what they timed.  Graph replays are repeated across several solves with
host work in between, so a replay that kept stale state would show."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

MODES = [
    ("whole graphs", dict(timing=abd.TIMING_OFF, use_graphs=1)),
    ("graphs, sampled PCG timing", dict(timing=abd.TIMING_PCG, use_graphs=1)),
    ("every stage timed", dict(timing=abd.TIMING_ALL)),
    ("direct launches", dict(timing=abd.TIMING_OFF, use_graphs=0)),
    ("direct, sampled PCG timing", dict(timing=abd.TIMING_PCG, use_graphs=0)),
    ("graphs, sampled assembly timing", dict(timing=abd.TIMING_ASM, use_graphs=1)),
]


def contact_spheres():
    return scenes.spheres_in_box_scene(
        3, n_bodies=24, level=1, half=0.25, y_lo=0.09, y_hi=0.45,
        r_lo=0.05, r_hi=0.08, min_gap=0.0005, vel=0.5, newton_theta=1e-7,
        pcg_eta=1e-12)


@pytest.mark.parametrize("name,mode", MODES, ids=[m[0] for m in MODES])
def test_launch_paths_match_oracle(name, mode):
    sc = contact_spheres()
    gpu = abd.Solver(sc)
    if "use_graphs" in mode:
        gpu.set_tuning(use_graphs=mode["use_graphs"])
    gpu.set_timing(mode["timing"])
    gpu.reset_timing()
    ref = O.Oracle(sc)
    newton = 0
    for k in range(8):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        sg = gpu.step()
        so = ref.step()
        assert sg["status"] == so["status"] == 0, (name, k)
        newton += sg["newton_iters"]
        err = np.abs(gpu.vertices() - ref.vertices()).max() / sg["scene_scale"]
        assert err < 1e-9, (name, k, err)
    tm = gpu.timing()
    if mode["timing"] == abd.TIMING_OFF:
        assert all(v["launches"] == 0 for v in tm.values())
    elif mode["timing"] == abd.TIMING_PCG:
        # a sample of the passes: at least one PCG launch per solve, fewer
        # than one per Newton iteration, and bytes for exactly those
        assert 2 <= tm["pcg"]["launches"] < newton
        assert tm["pcg"]["ms"] > 0.0 and tm["pcg"]["bytes"] >= 0.0
        assert all(v["launches"] == 0 for s, v in tm.items() if s != "pcg")
    elif mode["timing"] == abd.TIMING_ASM:
        # a sample of the passes' assembly launches, with their work
        assert 2 <= tm["assemble"]["launches"] < newton
        assert tm["assemble"]["ms"] > 0.0
        assert tm["assemble"]["bytes"] > 0.0 and tm["assemble"]["flops"] > 0.0
        assert all(v["launches"] == 0 for s, v in tm.items() if s != "assemble")
    else:
        assert tm["pcg"]["launches"] >= newton
        assert tm["broad"]["launches"] > 0 and tm["barrier"]["launches"] > 0
    gpu.close()

