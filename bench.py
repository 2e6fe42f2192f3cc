"""Benchmark of the local affine-body Newton solve on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 1000 level-3 icospheres (642 vertices, 1280 triangles each,
radius 0.05-0.15) at seeded non-overlapping positions falling into a
static open box; h = 0.01, dhat = 1e-3, kappa = 1e5, kappa_A = 1e8,
FP64, Newton tolerance 1e-6 (relative |dq|_inf / (h l)).  A step is one
time step (prediction, the full local Newton solve, commit); W steps run
untimed first, then K steps are timed.  value = Newton iterations per
second over the timed steps, inputs resident on the device throughout.

The JSON line carries the roofline of the dominant kernel (measured live
with HIP events on the library's stream) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel from two rocprofv3 --pmc runs of this
# benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each divided
# by what the same counter reads per byte for a plain device copy of known
# size (python bench.py --copy-probe).  Valid only for the kernel source it
# was measured on (sha256 of the PCG section of the kernel source);
# otherwise traffic is null.
PMC_TRAFFIC = {
    "kernel": "k_pcg_cg1<double>",
    "fetch_kib": 2473.1,       # FETCH_SIZE per dispatch, 90 dispatches
    "write_kib": 5346.0,       # WRITE_SIZE per dispatch, 90 dispatches
    "fetch_per_byte": 131086.5 / 262144.0,  # copy of 256 MiB reads 0.5
    "write_per_byte": 262144.0 / 262144.0,  # copy of 256 MiB writes 1.0
    "sha256": "6eaa85fabf0744a19da079fdfb0d3f500eee447519f4a32017c3fef0a441c2bb",
}

WORKLOAD = ("1000 icospheres (642 verts, 1280 tris each, r 0.05-0.15) "
            "falling into an open box container, dt 0.01, dhat 1e-3, "
            "kappa 1e5, kappa_A 1e8, FP64, Newton tol 1e-6")


def cpu_baseline(seed, n_steps):
    """Oracle on the first n_steps time steps of the same scene."""
    from oracle import oracle as O
    from paper_2605_15875_amd import scenes
    sc = scenes.config(1, seed)
    orc = O.Oracle(sc)
    iters = 0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        st = orc.step()
        iters += st["newton_iters"]
    dt = time.perf_counter() - t0
    return dict(value=iters / dt, unit="newton_iters/s", cores=1,
                kind="oracle",
                sample=f"first {n_steps} time steps of the workload "
                       f"({iters} Newton iterations, {dt:.1f} s, "
                       f"single thread)")


def copy_probe():
    """A plain device copy of known size, to calibrate the HBM counters."""
    import torch
    n = 256 << 20  # bytes per buffer
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 3}), flush=True)


def kernel_sha():
    """sha256 of the PCG section of the kernel source (the block-Jacobi PCG
    kernels and their helpers), which the traffic figures belong to."""
    import hashlib
    path = os.path.join(ROOT, "paper_2605_15875_amd", "csrc", "kernels.hip")
    with open(path, "r") as f:
        src = f.read()
    a = src.index("/* S7 block-Jacobi PCG")
    b = src.index("/* Single-reduction (pipelined) block-Jacobi PCG")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def pmc_traffic(kernel):
    t = PMC_TRAFFIC
    if not t or t["kernel"] != kernel or t["sha256"] != kernel_sha():
        return None
    return (t["fetch_kib"] * 1024.0 / t["fetch_per_byte"] +
            t["write_kib"] * 1024.0 / t["write_per_byte"])


def bench_batch(abd, scenes, torch, n_scenes, steps, warmup):
    """n_scenes independent 8-cube scenes (different seeds, same
    parameters): one batched solve per step against one solve per context
    in turn.  Both advance identical copies of the scenes."""
    import time as _t
    scs = [scenes.config(0, seed) for seed in range(n_scenes)]
    one = [abd.Solver(sc) for sc in scs]
    many = [abd.Solver(sc) for sc in scs]
    bt = abd.Batch(many)

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        it = 0
        for _ in range(steps):
            it += fn()
        torch.cuda.synchronize()
        return it, _t.perf_counter() - t0

    def seq():
        return sum(s.step()["newton_iters"] for s in one)

    def bat():
        return sum(st["newton_iters"] for st in bt.step())

    it_s, t_s = run(seq)
    it_b, t_b = run(bat)
    bt.close()
    for s in one + many:
        s.close()
    return dict(workload=f"{n_scenes} independent 8-cube scenes, FP64",
                steps=steps, batched_newton_iters_per_s=it_b / t_b,
                sequential_newton_iters_per_s=it_s / t_s,
                batched_ms_per_step=t_b * 1e3 / steps,
                sequential_ms_per_step=t_s * 1e3 / steps,
                speedup=(it_b / t_b) / (it_s / t_s))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--breakdown-steps", type=int, default=3)
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--pcg-variant", type=int, default=None,
                    help="0: two grid barriers per PCG iteration, "
                         "1: single-reduction form (default: library's)")
    ap.add_argument("--overlap-body", type=int, default=None,
                    help="1: body terms on a second stream, 0: in line")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library autotuner after warmup")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device copy of known size (counter "
                         "calibration) and exit")
    a = ap.parse_args()
    if a.copy_probe:
        copy_probe()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the local solve of one worker runs "
              "on a single device; multi-GPU runs are not part of this "
              "build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2605_15875_amd import abd, scenes
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    def log(*m):
        if not a.quiet:
            print(*m, file=sys.stderr, flush=True)

    sc = scenes.config(1, a.seed)
    log(f"scene: {len(sc.bodies)} bodies, {sc.n_vertices} verts, "
        f"{sc.n_triangles} tris")
    solver = abd.Solver(sc)
    if a.pcg_variant is not None:
        solver.set_tuning(pcg_variant=a.pcg_variant)
    if a.overlap_body is not None:
        solver.set_tuning(overlap_body=a.overlap_body)
    for i in range(a.warmup):
        st = solver.step()
        log(f"warmup {i}: newton={st['newton_iters']} "
            f"pcg={st['pcg_iters_total']} ms={st['t_solve_ms']:.1f}")
    if a.autotune:
        log(f"autotuned: {solver.autotune()}")
    tuning = solver.tuning()
    # timed region: the PCG launch of every fourth pass is bracketed by
    # events, so the PCG kernel's launch duration is measured on a sample of
    # the timed region's own launches
    solver.set_timing(abd.TIMING_PCG)
    solver.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = pcg = 0
    for i in range(a.steps):
        st = solver.step()
        newton += st["newton_iters"]
        pcg += st["pcg_iters_total"]
        log(f"step {i}: newton={st['newton_iters']} pcg={st['pcg_iters_total']}"
            f" active={st['n_active']} cand={st['n_cand_pt']}+"
            f"{st['n_cand_ee']} alpha_min={st['min_alpha']:.3g} "
            f"ms={st['t_solve_ms']:.1f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm_timed = solver.timing()
    x64 = solver.vertices()  # state after warmup + timed steps
    # stage breakdown from extra instrumented steps (every stage timed,
    # direct launches instead of graphs); not part of the timed region
    solver.set_timing(abd.TIMING_ALL)
    solver.reset_timing()
    for i in range(a.breakdown_steps):
        solver.step()
    tm = solver.timing()
    solver.set_timing(abd.TIMING_OFF)
    if not any(v["launches"] for v in tm.values()):
        tm = tm_timed
    # the dominant single kernel is the PCG solve (the broad-phase stage
    # sums several smaller kernels); its launches are timed with events in
    # the timed region itself
    dom = "pcg"
    roof = None
    d = tm_timed[dom]
    pcg_kernel = {abd.PCG_LOCAL: "k_pcg_local", abd.PCG_TWO_BARRIER: "k_pcg",
                  abd.PCG_PIPELINED: "k_pcg1",
                  abd.PCG_LOCAL1: "k_pcg_cg1"}[tuning["pcg_variant"]] + "<double>"
    if d["bytes"] > 0 and d["launches"]:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        kname = pcg_kernel if dom == "pcg" else dom
        traffic = pmc_traffic(kname)
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel=kname,
                    bytes_per_launch=d["bytes"] / d["launches"],
                    launches=d["launches"],
                    avg_launch_ms=d["ms"] / d["launches"],
                    measured="timed region" if dom == "pcg"
                    else "instrumented steps")
    l = float(np.linalg.norm(np.ptp(x64, axis=0)))
    mixed = None
    if not a.no_mixed:
        # same workload, same steps and tolerance, FP32 Hessian path
        ms = abd.Solver(sc, precision=1)
        ms.set_tuning(**tuning)
        for i in range(a.warmup):
            ms.step()
        ms.set_timing(abd.TIMING_PCG)  # same event overhead as FP64
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mnewton = fallbacks = 0
        for i in range(a.steps):
            st = ms.step()
            mnewton += st["newton_iters"]
            fallbacks += st["fp64_fallback"]
        torch.cuda.synchronize()
        mel = time.perf_counter() - t1
        xm = ms.vertices()
        # accuracy: time steps of both precisions from the same states (the
        # free-running trajectories of a contact pile branch apart once one
        # solve settles in a different local minimum)
        one_step = 0.0
        for i in range(3):
            q, qd = solver.get_state()
            ms.set_state(q, qd)
            solver.step()
            ms.step()
            one_step = max(one_step, float(
                np.abs(ms.vertices() - solver.vertices()).max() / l))
        mixed = dict(newton_iters_per_s=mnewton / mel, newton_iters=mnewton,
                     fp64_fallback_steps=fallbacks,
                     ms_per_step=mel * 1e3 / a.steps,
                     speedup_vs_fp64=elapsed / mel,
                     one_step_pos_diff_vs_fp64_over_l=one_step,
                     free_running_pos_diff_vs_fp64_over_l=float(
                         np.abs(xm - x64).max() / l))
        log(f"mixed: {mnewton} newton iters in {mel*1e3:.1f} ms")
        ms.close()
    solver.close()
    batch = None
    if not a.no_batch:
        batch = bench_batch(abd, scenes, torch, a.batch_scenes, 5, 1)
        log(f"batch: {batch}")
    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline ...")
        cpu = cpu_baseline(a.seed, a.cpu_steps)
    out = {
        "metric": "local Newton iters/s at ~1M tris",
        "value": newton / elapsed,
        "unit": "newton_iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "bodies": len(sc.bodies) - 1,
                   "triangles": sc.n_triangles, "vertices": sc.n_vertices,
                   "seed": a.seed, "precision": "fp64", "tuning": tuning},
        "newton_iters": newton,
        "pcg_iters": pcg,
        "stage_ms_instrumented": {k: round(v["ms"] / max(a.breakdown_steps, 1),
                                           3) for k, v in tm.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "mixed_vs_fp64_speedup": mixed["speedup_vs_fp64"] if mixed else None,
        "mixed": mixed,
        "batch": batch,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
