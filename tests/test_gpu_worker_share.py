"""One worker's share of an ADMM split (convex hulls in a funnel of static
walls, cut at x = 0): shared bodies carry consensus targets z = q~ + seeded
offsets, duals u, rho = 1e4 and kappa_b = 2, pairs use the by-shared-set
replication rule, and each time step runs several local solves (warm
started, as successive ADMM iterations call them) with z moved toward a
synthetic neighbour replica between them.  Each local solve is compared
with the oracle from the same start state."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import abd, scenes

pytestmark = pytest.mark.gpu


def share_scene():
    return scenes.hulls_in_funnel_scene(
        0, n_bodies=120, n_lo=40, n_hi=80, n_shared=20, newton_theta=1e-8,
        pcg_eta=1e-12)


def test_worker_share_local_solves_match_oracle():
    sc = share_scene()
    ids = sc.shared_ids
    n = len(ids)
    assert n >= 10
    gpu = abd.Solver(sc)
    ref = O.Oracle(sc, dense_max_dof=0)
    for s in (gpu, ref):
        s.set_pair_replication(1)
    rng = np.random.default_rng(11)
    for step in range(3):
        q, qd = ref.get_state()
        gpu.set_state(q, qd)
        gpu.begin_step()
        ref.begin_step()
        qt = ref.qtilde()
        z = qt[ids] + sc.shared_delta
        u = sc.shared_u.copy()
        for k in range(3):  # ADMM iterations: local solve, then new z, u
            for s in (gpu, ref):
                s.set_shared(ids, z, u, sc.shared_rho, sc.shared_kappa)
            sg = gpu.local_solve()
            so = ref.local_solve()
            assert sg["status"] == so["status"] == 0
            l = sg["scene_scale"]
            err = np.abs(gpu.vertices() - ref.vertices()).max() / l
            assert err < 1e-9, (step, k, err)
            # continue both from the oracle's iterate
            qo, _ = ref.get_state()
            gpu.set_state(qo)
            # synthetic neighbour replica: z averages the local block with a
            # seeded perturbation of it (Eq. 6 with equal rho), u per Eq. 7
            nb = qo[ids] + 0.5 ** (k + 1) * rng.uniform(-1e-4, 1e-4, (n, 12))
            z_new = 0.5 * ((qo[ids] + u) + (nb + u))
            u = u + qo[ids] - z_new
            z = z_new
        for s in (gpu, ref):
            s.end_step()
        nc, md = ref.penetration(ref.vertices())
        assert nc == 0 and md > 0
    gpu.close()
