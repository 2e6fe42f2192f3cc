"""Benchmark of the local affine-body Newton solve on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 1000 level-3 icospheres (642 vertices, 1280 triangles each,
radius 0.05-0.15) at seeded non-overlapping positions falling into a
static open box; h = 0.01, dhat = 1e-3, kappa = 1e5, kappa_A = 1e8,
FP64, Newton tolerance 1e-6 (relative |dq|_inf / (h l)).  A step is one
time step (prediction, the full local Newton solve, commit); W steps run
untimed first, then K steps are timed.  value = Newton iterations per
second over the timed steps, inputs resident on the device throughout.

Also on the line:
  roofline      the dominant kernel (the barrier assembly, k_assemble), its
                launch duration measured with HIP events on the library's
                stream inside the timed region (every fourth pass);
  roofline_s5   the barrier stage (distance filter and assembly) against
                both the HBM and the FP64 roofline, from extra steps with
                every stage timed;
  run50         all 50 steps of the workload from its initial state, FP64
                and mixed precision, each step checked for penetration on
                the device; mixed_vs_fp64_speedup is the ratio of their
                wall times;
  vs_oracle     per-step position errors of the FP64 and mixed GPU steps
                against the CPU oracle's steps from the same states (the
                first timed steps);
  cpu_baseline  the oracle (single thread) on those same time steps, and
                cpu_baseline_omp its OpenMP build on all host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

# HBM traffic of the dominant kernel from two rocprofv3 --pmc runs of this
# benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each divided
# by what the same counter reads per byte for a plain device copy of known
# size (python bench.py --copy-probe).  Valid only for the kernel source it
# was measured on (sha256 of the kernel's section of the kernel source);
# otherwise traffic is null.
PMC_TRAFFIC = {
    "kernel": "k_assemble<double>",
    "section": ("/* S5 barrier: narrow phase filter and assembly",
                "/* S7 block-Jacobi PCG"),
    "fetch_kib": 441.96,       # FETCH_SIZE per dispatch, 91 dispatches
    "write_kib": 322.5,        # WRITE_SIZE per dispatch, 91 dispatches
    "fetch_per_byte": 131086.77 / 262144.0,  # copy of 256 MiB reads 0.5
    "write_per_byte": 262144.0 / 262144.0,  # copy of 256 MiB writes 1.0
    "sha256": "c147b8b6b6ae0f2818e3e3d1a71e5e8307c04fc8cd784f95831cf938f27f5506",
}

METRIC = ("local Newton iters/s at ~1M tris; mixed vs FP64 speedup at 1e-6 "
          "residual")
WORKLOAD = ("1000 icospheres (642 verts, 1280 tris each, r 0.05-0.15) "
            "falling into an open box container, dt 0.01, dhat 1e-3, "
            "kappa 1e5, kappa_A 1e8, FP64, Newton tol 1e-6")


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def step(solver):
    """One time step; a solve that ends without convergence (NOCONV) keeps
    its last iterate, which is penetration free like every iterate, and the
    step is counted as such instead of stopping the benchmark."""
    solver.begin_step()
    st = solver.local_solve(check=False)
    if st["status"] not in (0, -4):
        raise RuntimeError(f"local solve failed: status {st['status']}: "
                           f"{solver.error()}")
    solver.end_step()
    return st


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


def kernel_sha(section):
    """sha256 of a section of the kernel source (between two banner
    comments), which a kernel's traffic figures belong to."""
    import hashlib
    path = os.path.join(ROOT, "paper_2605_15875_amd", "csrc", "kernels.hip")
    with open(path, "r") as f:
        src = f.read()
    a = src.index(section[0])
    b = src.index(section[1])
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def pmc_traffic(kernel):
    t = PMC_TRAFFIC
    if (not t or t["kernel"] != kernel or t["sha256"] is None or
            t["sha256"] != kernel_sha(t["section"])):
        return None
    return (t["fetch_kib"] * 1024.0 / t["fetch_per_byte"] +
            t["write_kib"] * 1024.0 / t["write_per_byte"])


def run_all_steps(abd, sc, n, precision, tuning, log):
    """All n steps from the initial state: wall time of the steps alone,
    every state checked for penetration on the device between steps."""
    s = abd.Solver(sc, precision=precision)
    s.set_tuning(**tuning)
    t = 0.0
    newton = n32 = switched = noconv = 0
    worst_newton = 0
    min_dist = float("inf")
    crossings = 0
    for k in range(n):
        t0 = time.perf_counter()
        st = step(s)
        t += time.perf_counter() - t0
        newton += st["newton_iters"]
        n32 += st["newton_fp32"]
        switched += st["fp64_fallback"]
        noconv += st["status"] == -4
        worst_newton = max(worst_newton, st["newton_iters"])
        nc, md = s.check_penetration()
        crossings += nc
        min_dist = min(min_dist, md)
    x = s.vertices()
    s.close()
    log(f"run{n} precision={precision}: {newton} newton in {t*1e3:.1f} ms, "
        f"switched={switched} noconv={noconv} min_dist={min_dist:.3g}")
    out = dict(steps=n, wall_ms=t * 1e3, newton_iters=newton,
               newton_iters_per_s=newton / t, max_newton_per_step=worst_newton,
               noconv_steps=noconv, penetration_free=bool(
                   crossings == 0 and min_dist > 0),
               edge_triangle_crossings=crossings, min_distance=min_dist)
    if precision:
        out.update(newton_fp32=n32, fp64_switch_steps=switched)
    return out, x


def versus_oracle(abd, O, sc, q0, qd0, n, gpu64, gpumx, log):
    """The oracle (single thread, then its OpenMP build) on n time steps
    from the state (q0, qd0); the FP64 and mixed GPU contexts step from the
    oracle's state before each of its steps, and their positions are
    compared with the oracle's after it."""
    import numpy as np
    ref = O.Oracle(sc)
    ref.set_state(q0, qd0)
    err64 = []
    errmx = []
    t_orc = 0.0
    it_orc = 0
    for k in range(n):
        q, qd = ref.get_state()
        for g in (gpu64, gpumx):
            g.set_state(q, qd)
        s64 = step(gpu64)
        smx = step(gpumx)
        t0 = time.perf_counter()
        sr = ref.step()
        t_orc += time.perf_counter() - t0
        it_orc += sr["newton_iters"]
        xr = ref.vertices()
        l = sr["scene_scale"]
        err64.append(float(np.abs(gpu64.vertices() - xr).max() / l))
        errmx.append(float(np.abs(gpumx.vertices() - xr).max() / l))
        log(f"oracle step {k}: newton={sr['newton_iters']} (gpu fp64 "
            f"{s64['newton_iters']}, mixed {smx['newton_iters']}) "
            f"err/l fp64={err64[-1]:.2e} mixed={errmx[-1]:.2e}")
    q_end, _ = ref.get_state()
    # the OpenMP build on the same steps (same results, several threads)
    omp = O.Oracle(sc, omp=True)
    omp.set_state(q0, qd0)
    t_omp = 0.0
    it_omp = 0
    for k in range(n):
        t0 = time.perf_counter()
        it_omp += omp.step()["newton_iters"]
        t_omp += time.perf_counter() - t0
    q_omp, _ = omp.get_state()
    same = bool(np.array_equal(q_end, q_omp))
    return (dict(steps=n, pos_err_over_l_fp64=err64,
                 pos_err_over_l_mixed=errmx, max_fp64=max(err64),
                 max_mixed=max(errmx)),
            dict(t=t_orc, it=it_orc), dict(t=t_omp, it=it_omp, same=same))


def bench_batch(abd, scenes, torch, n_scenes, steps, warmup):
    """n_scenes independent 8-cube scenes (different seeds, same
    parameters): one batched solve per step against one solve per context
    in turn.  Both advance identical copies of the scenes."""
    scs = [scenes.config(0, seed) for seed in range(n_scenes)]
    one = [abd.Solver(sc) for sc in scs]
    many = [abd.Solver(sc) for sc in scs]
    bt = abd.Batch(many)

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = 0
        for _ in range(steps):
            it += fn()
        torch.cuda.synchronize()
        return it, time.perf_counter() - t0

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


def bench_batch_workload(abd, scenes, torch, steps, log):
    """The batch workload: 8 ADMM subdomains of 200-3000 bodies (icospheres
    and hulls, each with its shared bodies and consensus data) and 64 cube
    scenes of 16-512 cubes, 6.8M triangles, solved together in the same
    launches (FP64 and mixed precision) against one context after another
    (FP64); the first `steps` time steps from the initial state.  Newton
    iterations are summed over the problems; a problem that ends a step
    without converging is counted, not dropped."""
    scs = scenes.batch_workload(0)

    def contexts(prec):
        out = [abd.Solver(sc, precision=prec) for sc in scs]
        for s in out:
            s.set_pair_replication(abd.PAIRS_BY_SHARED)
        return out

    def begin(ctxs):
        for sc, g in zip(scs, ctxs):
            g.begin_step()
            if sc.shared_ids is not None:
                z = g.qtilde()[sc.shared_ids] + sc.shared_delta
                g.set_shared(sc.shared_ids, z, sc.shared_u, sc.shared_rho,
                             sc.shared_kappa)

    def run(ctxs, solve):
        it, t, bad, per = 0, 0.0, 0, []
        for _ in range(steps):
            begin(ctxs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            for g in ctxs:
                g.end_step()
            n = sum(x["newton_iters"] for x in st)
            it += n
            t += dt
            bad += sum(1 for x in st if x["status"] != 0)
            per.append((round(dt * 1e3, 1), n))
        return dict(newton_iters_per_s=it / t, newton_iters=it,
                    ms_per_step=t * 1e3 / steps, unconverged_problem_steps=bad,
                    per_step_ms_and_iters=per)

    res = {}
    for name, prec in (("batched_fp64", 0), ("batched_mixed", 1)):
        ctxs = contexts(prec)
        bt = abd.Batch(ctxs)
        res[name] = run(ctxs, lambda: bt.local_solve(check=False))
        log(f"batch workload {name}: {res[name]}")
        bt.close()
        for g in ctxs:
            g.close()
    ctxs = contexts(0)
    res["sequential_fp64"] = run(
        ctxs, lambda: [g.local_solve(check=False) for g in ctxs])
    log(f"batch workload sequential_fp64: {res['sequential_fp64']}")
    for g in ctxs:
        g.close()
    res.update(
        workload=f"{len(scs)} problems: 8 ADMM subdomains of "
                 f"{min(scenes.BATCH_SUBDOMAINS)}-{max(scenes.BATCH_SUBDOMAINS)} "
                 f"bodies (icospheres and hulls) and 64 cube scenes of "
                 f"{min(scenes.BATCH_CUBES)}-{max(scenes.BATCH_CUBES)} cubes",
        bodies=sum(sc.n_dynamic for sc in scs),
        triangles=sum(sc.n_triangles for sc in scs), steps=steps,
        speedup_fp64=res["batched_fp64"]["newton_iters_per_s"]
        / res["sequential_fp64"]["newton_iters_per_s"],
        mixed_vs_fp64_wall=res["batched_fp64"]["ms_per_step"]
        / res["batched_mixed"]["ms_per_step"])
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="time steps of the oracle comparison and CPU "
                         "baseline (the first timed steps)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-run50", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="bit-reproducible solves (exact sums)")
    ap.add_argument("--max-ls", type=int, default=None,
                    help="line-search halvings (scene default if unset)")
    ap.add_argument("--run-steps", type=int, default=50)
    ap.add_argument("--breakdown-steps", type=int, default=3)
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-workload", action="store_true",
                    help="also run the batch workload leg (72 problems, "
                         "6.8M triangles; off by default)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-workload-only", action="store_true",
                    help="only the batch workload leg (its JSON on stdout)")
    ap.add_argument("--pcg-variant", type=int, default=None)
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

    import torch
    from paper_2605_15875_amd import abd, scenes
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    def log(*m):
        if not a.quiet:
            print(*m, file=sys.stderr, flush=True)

    if a.batch_workload_only:
        print(json.dumps(bench_batch_workload(abd, scenes, torch, a.batch_steps, log)),
              flush=True)
        return

    over = {}
    if a.deterministic:
        over["deterministic"] = 1
    if a.max_ls is not None:
        over["max_ls"] = a.max_ls
    sc = scenes.config(1, a.seed, **over)
    log(f"scene: {len(sc.bodies)} bodies, {sc.n_vertices} verts, "
        f"{sc.n_triangles} tris")
    solver = abd.Solver(sc)
    if a.pcg_variant is not None:
        solver.set_tuning(pcg_variant=a.pcg_variant)
    for i in range(a.warmup):
        st = step(solver)
        log(f"warmup {i}: newton={st['newton_iters']} "
            f"pcg={st['pcg_iters_total']} ms={st['t_solve_ms']:.1f}")
    if a.autotune:
        log(f"autotuned: {solver.autotune()}")
    tuning = solver.tuning()
    q_first, qd_first = solver.get_state()  # state at the first timed step
    # timed region: the assembly launch of every fourth pass (the dominant
    # kernel) is bracketed by events, so its launch duration is measured on
    # a sample of the timed region's own launches
    solver.set_timing(abd.TIMING_ASM)
    solver.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = pcg = noconv = 0
    per_step = []
    for i in range(a.steps):
        ts = time.perf_counter()
        st = step(solver)
        per_step.append((st["newton_iters"], time.perf_counter() - ts))
        newton += st["newton_iters"]
        pcg += st["pcg_iters_total"]
        noconv += st["status"] == -4
        log(f"step {i}: newton={st['newton_iters']} pcg={st['pcg_iters_total']}"
            f" active={st['n_active']} cand={st['n_cand_pt']}+"
            f"{st['n_cand_ee']} alpha_min={st['min_alpha']:.3g} "
            f"status={st['status']} ms={st['t_solve_ms']:.1f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm_timed = solver.timing()
    # stage breakdown from extra instrumented steps (every stage timed);
    # not part of the timed region
    solver.set_timing(abd.TIMING_ALL)
    solver.reset_timing()
    for i in range(a.breakdown_steps):
        step(solver)
    tm = solver.timing()
    solver.set_timing(abd.TIMING_OFF)
    if not any(v["launches"] for v in tm.values()):
        tm = tm_timed
    roof = None
    d = tm_timed["assemble"]
    if d["bytes"] > 0 and d["launches"]:
        # HBM-nominal (about 3 flops per algorithmic byte, below the FP64
        # ridge of 9.8); its FP64 fraction rides along
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        tfs = d["flops"] / (d["ms"] * 1e-3) / 1e12
        kname = "k_assemble<double>"
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=pmc_traffic(kname), kernel=kname,
                    bytes_per_launch=d["bytes"] / d["launches"],
                    flops_per_launch=d["flops"] / d["launches"],
                    fp64_achieved_TFs=tfs, fp64_frac=tfs / FP64_PEAK_TFS,
                    launches=d["launches"],
                    avg_launch_ms=d["ms"] / d["launches"],
                    measured="timed region, every fourth pass")
    roof5 = None
    d5 = tm["barrier"]
    if d5["launches"] and d5["ms"] > 0:
        gbs = d5["bytes"] / (d5["ms"] * 1e-3) / 1e9
        tfs = d5["flops"] / (d5["ms"] * 1e-3) / 1e12
        fh, ff = gbs / HBM_PEAK_GBS, tfs / FP64_PEAK_TFS
        roof5 = dict(bound="fp64" if ff > fh else "hbm",
                     kernels="k_filter + k_assemble<double>",
                     achieved_GBs=gbs, peak_GBs=HBM_PEAK_GBS, frac_hbm=fh,
                     achieved_TFs=tfs, peak_TFs=FP64_PEAK_TFS, frac_fp64=ff,
                     bytes_per_pass=d5["bytes"] / d5["launches"],
                     flops_per_pass=d5["flops"] / d5["launches"],
                     avg_ms_per_pass=d5["ms"] / d5["launches"],
                     passes=d5["launches"], traffic=None,
                     measured=f"{a.breakdown_steps} steps after the timed "
                              "region, every stage timed")
    solver.close()

    run50 = None
    mixed_speedup = None
    if not a.no_run50:
        r64, _ = run_all_steps(abd, sc, a.run_steps, 0, tuning, log)
        rmx, _ = run_all_steps(abd, sc, a.run_steps, 1, tuning, log)
        mixed_speedup = r64["wall_ms"] / rmx["wall_ms"]
        run50 = dict(workload=f"all {a.run_steps} steps from the initial "
                              "state", fp64=r64, mixed=rmx,
                     mixed_vs_fp64_wall_speedup=mixed_speedup)

    vs_oracle = cpu = cpu_omp = None
    if not a.no_cpu_baseline and a.cpu_steps > 0:
        from oracle import oracle as O
        log("oracle on the first timed steps ...")
        g64 = abd.Solver(sc)
        gmx = abd.Solver(sc, precision=1)
        for g in (g64, gmx):
            g.set_tuning(**tuning)
        vs_oracle, orc, omp = versus_oracle(abd, O, sc, q_first, qd_first,
                                            a.cpu_steps, g64, gmx, log)
        g64.close()
        gmx.close()
        n = a.cpu_steps
        gpu_it = sum(p[0] for p in per_step[:n])
        gpu_t = sum(p[1] for p in per_step[:n])
        sample = (f"time steps {a.warmup}-{a.warmup + n - 1} of the workload "
                  f"(the first {n} timed steps) from the GPU's state at the "
                  f"first timed step: {orc['it']} Newton iterations")
        cpu = dict(value=orc["it"] / orc["t"], unit="newton_iters/s", cores=1,
                   kind="oracle", sample=sample + f", {orc['t']:.1f} s",
                   gpu_same_steps_newton_iters_per_s=gpu_it / gpu_t)
        cpu_omp = dict(value=omp["it"] / omp["t"], unit="newton_iters/s",
                       cores=host_cores(), kind="oracle (OpenMP build)",
                       sample=sample + f", {omp['t']:.1f} s",
                       bit_identical_to_single_thread=omp["same"])
    batch = None
    if not a.no_batch:
        batch = bench_batch(abd, scenes, torch, a.batch_scenes, 5, 1)
        log(f"batch: {batch}")
    batch_wl = None
    if a.batch_workload:
        batch_wl = bench_batch_workload(abd, scenes, torch, a.batch_steps, log)
    out = {
        "metric": METRIC,
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
        "noconv_steps": noconv,
        "stage_ms_instrumented": {k: round(v["ms"] / max(a.breakdown_steps, 1),
                                           3) for k, v in tm.items()},
        "roofline": roof,
        "roofline_s5": roof5,
        "cpu_baseline": cpu,
        "cpu_baseline_omp": cpu_omp,
        "host_cores": host_cores(),
        "mixed_vs_fp64_speedup": mixed_speedup,
        "run50": run50,
        "vs_oracle": vs_oracle,
        "batch": batch,
        "batch_workload": batch_wl,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
