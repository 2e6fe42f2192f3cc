"""The batch workload: ADMM subdomains of uneven size (icospheres and
convex hulls, each with shared bodies and consensus data) and independent
cube scenes, solved together in the same launches.

Reduced size, with the launch paths of large batches forced on a small
one: body pairs by sort and sweep, component labels per chunk of whole
problems after the three-kernel block-row build, and the problem-local
PCG in several launches; every problem against the oracle's solve of it
alone, in lock-step.  Full size (8 subdomains of 200-3000 bodies, 64 cube
scenes of 16-512 cubes, 6.8M triangles, the launch configuration the
benchmark times): two batched steps, every problem converged and
penetration free, and sampled problems against the oracle from the same
state."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu

SMALL = dict(subdomains=(14, 30), cubes=(4, 9, 16),
             sub_args=dict(level=1, n_lo=20, n_hi=40, width=1.2))


def _begin(scs, gpus, refs):
    """Start a step on both sides from the oracle's state; consensus
    targets from the oracle's prediction."""
    for sc, g, r in zip(scs, gpus, refs):
        q, qd = r.get_state()
        g.set_state(q, qd)
        g.begin_step()
        r.begin_step()
        if sc.shared_ids is not None:
            z = r.qtilde()[sc.shared_ids] + sc.shared_delta
            for s in (g, r):
                s.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho,
                             sc.shared_kappa)


@pytest.mark.parametrize("precision", [0, 1])
def test_small_batch_workload_forced_paths_match_oracle(precision):
    scs = scenes.batch_workload(6, newton_theta=1e-7, pcg_eta=1e-12,
                                precision=precision, **SMALL)
    refs = [O.Oracle(sc, dense_max_dof=0) for sc in scs]
    gpus = [abd.Solver(sc) for sc in scs]
    for s in gpus + refs:
        s.set_pair_replication(1)
    gpus[0].set_tuning(body_pairs=abd.BODY_PAIRS_SWEEP, pcg_launch_groups=2,
                       label_rows=48)
    bt = abd.Batch(gpus)
    active = 0
    for step in range(13):
        _begin(scs, gpus, refs)
        stats = bt.local_solve()
        for i, (g, r) in enumerate(zip(gpus, refs)):
            so = r.local_solve()
            active += so["n_active"]
            assert stats[i]["status"] == so["status"] == 0, (step, i)
            l = stats[i]["scene_scale"]
            err = np.abs(g.vertices() - r.vertices()).max() / l
            assert err < 1e-9, (step, i, err)
            g.set_state(*r.get_state())
            g.end_step()
            r.end_step()
    # contacts formed in every kind of problem
    assert active > 0
    bt.close()


def test_small_batch_workload_paths_agree():
    """Every pair of launch paths gives the same steps: forced sort and
    sweep with chunked labels and split PCG launches against the default
    all-pairs, one-workgroup paths."""
    scs = scenes.batch_workload(6, newton_theta=1e-7, pcg_eta=1e-12, **SMALL)
    a = [abd.Solver(sc) for sc in scs]
    b = [abd.Solver(sc) for sc in scs]
    for s in a + b:
        s.set_pair_replication(1)
    b[0].set_tuning(body_pairs=abd.BODY_PAIRS_SWEEP, pcg_launch_groups=2,
                    label_rows=48)
    ba, bb = abd.Batch(a), abd.Batch(b)
    for step in range(13):
        scale = None
        for bt, ss in ((ba, a), (bb, b)):
            for sc, s in zip(scs, ss):
                s.begin_step()
                if sc.shared_ids is not None:
                    z = s.qtilde()[sc.shared_ids] + sc.shared_delta
                    s.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho,
                                 sc.shared_kappa)
            st = bt.local_solve()
            assert all(x["status"] == 0 for x in st), step
            scale = scale or [x["scene_scale"] for x in st]
            for s in ss:
                s.end_step()
        for i, (x, y) in enumerate(zip(a, b)):
            err = np.abs(x.vertices() - y.vertices()).max() / scale[i]
            assert err < 1e-9, (step, i, err)
            y.set_state(*x.get_state())
    ba.close()
    bb.close()


def test_full_batch_workload():
    scs = scenes.batch_workload(0, newton_theta=1e-7, pcg_eta=1e-12)
    nb = sum(sc.n_dynamic for sc in scs)
    nt = sum(sc.n_triangles for sc in scs)
    assert len(scs) == 72 and nb > 15000 and nt > 6_000_000
    gpus = [abd.Solver(sc) for sc in scs]
    for s in gpus:
        s.set_pair_replication(1)
    bt = abd.Batch(gpus)
    sample = [0, 8, 71]  # the 200-body subdomain, 16 and 512 cubes
    refs = {}
    for step in range(2):
        for sc, g in zip(scs, gpus):
            g.begin_step()
            if sc.shared_ids is not None:
                z = g.qtilde()[sc.shared_ids] + sc.shared_delta
                g.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho,
                             sc.shared_kappa)
        if step == 1:
            # the oracle from the GPU's state at the start of this step
            for i in sample:
                q, qd = gpus[i].get_state()
                r = O.Oracle(scs[i], dense_max_dof=0, omp=True)
                r.set_pair_replication(1)
                r.set_state(q, qd)
                r.begin_step()
                if scs[i].shared_ids is not None:
                    z = r.qtilde()[scs[i].shared_ids] + scs[i].shared_delta
                    r.set_shared(scs[i].shared_ids, z, scs[i].shared_u,
                                 scs[i].shared_rho, scs[i].shared_kappa)
                refs[i] = r
        t0 = time.perf_counter()
        stats = bt.local_solve()
        ms = (time.perf_counter() - t0) * 1e3
        print(f"batched step {step}: {ms:.1f} ms, "
              f"{sum(st['newton_iters'] for st in stats)} Newton iterations "
              f"over {len(stats)} problems", flush=True)
        assert all(st["status"] == 0 for st in stats), step
        if step == 1:
            for i in sample:
                so = refs[i].local_solve()
                assert so["status"] == 0
                l = stats[i]["scene_scale"]
                err = np.abs(gpus[i].vertices() - refs[i].vertices()).max() / l
                print(f"problem {i}: newton {stats[i]['newton_iters']} vs "
                      f"{so['newton_iters']}, position error / l = {err:.2e}")
                assert err < 1e-9, (i, err)
        for g in gpus:
            g.end_step()
    for i, g in enumerate(gpus):
        nc, md = g.check_penetration()
        assert nc == 0 and md > 0, i
    bt.close()
