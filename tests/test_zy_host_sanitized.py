"""The host runtime under UndefinedBehaviorSanitizer: libabd_san.so (the
library with its host code built with -fsanitize=undefined, every report
fatal) drives contexts through finalize, solves, tuning changes that
switch to sort and sweep, chunked component labels and split PCG
launches, the hooks, a batch, the deterministic and mixed modes and the
allocation-free solve, in a child process with the UBSan runtime
preloaded.  (The AddressSanitizer runtime of this toolchain intercepts the
HSA allocator and fails its first device allocation, so the host runtime
has no ASan run; the oracle has one, tests/test_oracle_sanitized.py.)
It is collected after the other GPU parity tests, since unlike them it
depends on the process environment (the preloaded runtime)."""
import glob
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from paper_2605_15875_amd import abd, scenes
sc = scenes.cubes_scene(0, 2, 2, 2)
g = abd.Solver(sc)
for _ in range(12):
    assert g.step()["status"] == 0
g.set_tuning(body_pairs=abd.BODY_PAIRS_SWEEP, pcg_launch_groups=1, label_rows=4)
for _ in range(4):
    assert g.step()["status"] == 0
q, qd = g.get_state()
g.begin_step()
x = g.vertices()
pt = g.candidates(0); ee = g.candidates(1)
e = g.eval(); dq, _ = g.direction(); a, toi = g.ccd(dq, per_pair=True); g.energy_delta(dq, a)
g.check_penetration()
g.local_solve(); g.end_step()
scs = [scenes.cubes_scene(s, 2, 1, 2) for s in range(3)]
ctx = [abd.Solver(s) for s in scs]
bt = abd.Batch(ctx)
for _ in range(6):
    assert all(s["status"] == 0 for s in bt.step())
bt.close()
d = abd.Solver(scenes.cubes_scene(1, 2, 2, 2, deterministic=1))
for _ in range(12):
    assert d.step()["status"] == 0
m = abd.Solver(scenes.cubes_scene(1, 2, 2, 2, precision=1))
for _ in range(12):
    assert m.step()["status"] == 0
s2 = abd.Solver(scenes.cubes_scene(2, 2, 2, 2))
for _ in range(3):
    s2.begin_step(); s2.local_solve_static(); s2.end_step()
for h in [g, d, m, s2] + ctx:
    h.close()
print("sanitized host runtime ok", flush=True)
"""


def test_host_runtime_under_ubsan():
    lib = os.path.join(ROOT, "paper_2605_15875_amd", "libabd_san.so")
    if not os.path.exists(lib):
        pytest.skip("libabd_san.so not built")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/"
                          "libclang_rt.ubsan_standalone-x86_64.so"))
    if not rt:
        pytest.skip("no UBSan runtime")
    # the UBSan runtime is added after whatever the environment already
    # preloads, which stays preloaded as it is
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, LD_PRELOAD=(pre + ":" if pre else "") + rt[-1], ABD_LIB=lib,
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-u", "-c", SCRIPT], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    report = r.stdout[-2000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr, report
    assert "sanitized host runtime ok" in r.stdout, report
