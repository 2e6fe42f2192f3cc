"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
a sanitized build drives a cube stack, a hull worker share with its
consensus penalty, and the hooks (candidates, system, direction, CCD,
exact TOI, energy difference, penetration check) in a child process with
the sanitizer runtime preloaded; any report fails the test."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = r"""
import numpy as np
from oracle import oracle as O
from paper_2605_15875_amd import scenes
sc = scenes.cubes_scene(0, 2, 2, 2)
r = O.Oracle(sc)
for _ in range(12):
    assert r.step()["status"] == 0
sc = scenes.hulls_in_funnel_scene(0, n_bodies=40, n_lo=20, n_hi=40, n_shared=6)
r = O.Oracle(sc, dense_max_dof=0)
r.set_pair_replication(1)
for _ in range(3):
    r.begin_step()
    z = r.qtilde()[sc.shared_ids] + sc.shared_delta
    r.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho, sc.shared_kappa)
    assert r.local_solve()["status"] == 0
    r.end_step()
q, _ = r.get_state()
r.begin_step()
x = r.vertices()
for kind in (O.PT, O.EE):
    r.candidates(kind, x)
e = r.eval(q)
dq, _ = r.direction(q)
a = r.ccd(q, dq)
r.energy_delta(q, dq, a)
r.penetration(x)
xx = np.array([0.0, 1.0, 0.0, -1.0, 0.0, -1.0, 1.0, 0.0, -1.0, 0.0, 0.0, 1.0])
dx = np.zeros(12); dx[1] = -2.0
O.exact_toi(O.PT, xx, dx)
O.accd(O.PT, xx, dx, 0.1, 1.0)
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"],
                          capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no libasan for g++")
    from oracle import build
    lib = build.build_sanitized()
    # the sanitizer runtime goes first; whatever the environment already
    # preloads stays preloaded after it
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, LD_PRELOAD=asan + (":" + pre if pre else ""), ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr, report
    assert "runtime error" not in r.stderr, report
    assert "sanitized oracle ok" in r.stdout
