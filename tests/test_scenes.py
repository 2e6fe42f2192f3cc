"""Inputs of the batch workload: problem structure, shared parameters, the
shared bodies at the cut planes, and a feasible start that the oracle
steps from."""
import numpy as np

from oracle import oracle as O
from paper_2605_15875_amd import scenes


def test_batch_workload_structure():
    scs = scenes.batch_workload(0)
    subs, cubes = scs[:8], scs[8:]
    assert [s.n_dynamic for s in subs] == list(scenes.BATCH_SUBDOMAINS)
    assert [s.n_dynamic for s in cubes] == list(scenes.BATCH_CUBES)
    assert min(scenes.BATCH_SUBDOMAINS) == 200 and max(scenes.BATCH_SUBDOMAINS) == 3000
    assert min(scenes.BATCH_CUBES) == 16 and max(scenes.BATCH_CUBES) == 512
    assert 6_000_000 < sum(s.n_triangles for s in scs) < 7_500_000
    # one batch needs one parameter set
    assert all(s.params == scs[0].params for s in scs)
    for s in subs:
        tris = [len(b.tris) for b in s.bodies if b.kind == scenes.DYNAMIC]
        assert min(tris) >= 596 and max(tris) <= 2396
        ids = s.shared_ids
        assert len(ids) == round(0.1 * s.n_dynamic)
        # the shared bodies are those nearest the cut planes x = 0 and x = 4
        x = np.array([b.q0[0] for b in s.bodies if b.kind == scenes.DYNAMIC])
        edge = np.minimum(x, 4.0 - x)
        assert edge[ids].max() <= np.delete(edge, ids).min()
    for s in cubes:
        assert s.shared_ids is None and len(s.bodies) == s.n_dynamic + 1


def test_small_batch_workload_steps_on_the_oracle():
    scs = scenes.batch_workload(6, newton_theta=1e-6, subdomains=(14, 30),
                                cubes=(4, 9),
                                sub_args=dict(level=1, n_lo=20, n_hi=40,
                                              width=1.2))
    for sc in scs:
        r = O.Oracle(sc, dense_max_dof=0)
        r.set_pair_replication(1)
        for _ in range(3):
            r.begin_step()
            if sc.shared_ids is not None:
                z = r.qtilde()[sc.shared_ids] + sc.shared_delta
                r.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho,
                             sc.shared_kappa)
            assert r.local_solve()["status"] == 0
            r.end_step()
        nc, md = r.penetration(r.vertices())
        assert nc == 0 and md > 0
