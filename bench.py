"""Throughput of the DFSPH time step on one MI355X.

One step = sph_build_neighbors + sph_step (grid sort, neighbour lists, density
and alpha, divergence-free solve, non-pressure forces, warm start,
constant-density solve, rigid coupling, integration) on a synthetic scene
already resident in HBM.  Prints one JSON line.

Each arm runs --prerun untimed steps from the scene's start, then --warmup
steps (the last five time every kernel with HIP events), then --reps
repetitions of exactly --steps timed steps, each bracketed by a device
synchronisation; the reported throughput is the median repetition's.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5|c2|c3|c4|c1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s

# per-launch algorithmic bytes are computed inside the library (see the
# design notes: own fields of every particle read/written once plus 4 B per
# neighbour-list entry)
PROFILED = ("pressure_update", "predict", "density_alpha", "xsph", "nbr_build", "sort", "integrate", "visc",
            "warm_features", "mlp", "eos")
KERNEL_SOURCES = ("sph_kernels.hip", "sph_device.h", "sph_internal.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="steps of the benchmark workload the all-cores oracle runs for the CPU baseline")
    ap.add_argument("--prerun", type=int, default=100,
                    help="untimed steps before the warmup, so that the timed window is past the start-up transient")
    ap.add_argument("--reps", type=int, default=3,
                    help="repetitions of the timed window; the reported figure is their median")
    ap.add_argument("--arm", choices=("plain", "learned", "both"), default="both",
                    help="warm start of the density solve: previous-step (plain) and/or the trained MLP")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def kernel_sha() -> str:
    """Digest of the kernel sources, to tie counter runs to the code they measured."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2403_11156_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(config: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (scaled FETCH_SIZE + WRITE_SIZE), or None if they were taken on a
    different kernel source than the one built now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{config}.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_sha()
    table, recorded = {}, None
    for line in open(path):
        parts = line.split()
        if not parts or parts[0].startswith("#"):
            continue
        if parts[0] == "source_sha":
            recorded = parts[1]
        elif len(parts) == 3:
            table[parts[0]] = int(parts[1]) + int(parts[2])
    if recorded != sha:
        return None
    return table.get(kernel)


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable, os.cpu_count() or usable


def _oracle_rate(O, scene, steps, openmp):
    O.use_openmp(openmp)
    try:
        st = O.State(scene)
        t0 = time.perf_counter()
        for _ in range(steps):
            out = O.step(st)
            st = O.advance(st, out)
        dt = time.perf_counter() - t0
    finally:
        O.use_openmp(False)
    return scene.n_fluid * steps / dt, dt


def cpu_baseline(scene_name: str, steps: int):
    """The FP64 oracle, as it stands, on the host's cores: `steps` steps of
    the benchmark workload from its initial state on all usable cores
    (OpenMP over the independent per-particle loops, reductions in a fixed
    order, the same results as one thread), one step of it on one thread,
    and the small dam break (c1) over all its 100 steps both ways."""
    from oracle import oracle as O
    from paper_2403_11156_amd import scenes
    O.build(force=False)
    O.build(force=False, openmp=True)
    model, usable, total = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", usable))
    sc = scenes.scene(scene_name)
    v_all, t_all = _oracle_rate(O, sc, steps, True)
    v_one, t_one = _oracle_rate(O, sc, 1, False)
    c1 = scenes.scene("c1")
    c1_all, c1_t_all = _oracle_rate(O, c1, 100, True)
    c1_one, c1_t_one = _oracle_rate(O, c1, 100, False)
    return {"value": v_all, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} step(s) of {sc.name} from its initial state, FP64, {threads} OpenMP threads, "
                      f"{t_all:.1f} s",
            "host": {"cpu_model": model, "usable_cores": usable, "logical_cpus": total},
            "one_thread": {"value": v_one, "sample": f"1 step of {sc.name}, FP64, 1 thread, {t_one:.1f} s"},
            "c1_100_steps": {"all_cores": c1_all, "one_thread": c1_one,
                             "seconds": {"all_cores": round(c1_t_all, 2), "one_thread": round(c1_t_one, 2)}}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs the step on one GPU only (--gpus 1)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2403_11156_amd import scenes, sph

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        # a read-only pass over the same bytes (a sum): a second kernel of
        # known traffic for the read counter
        total = float(b.sum())
        print(f"[bench] calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB written; "
              f"then a sum reading {args.calib_copy_mb} MiB ({total:.0f})", flush=True)
        del a, b
    sc = scenes.scene(args.config)
    weights = os.path.join(ROOT, "paper_2403_11156_amd", "weights", "warm_start_mlp.f32")
    solver = sc.params.get("solver", scenes.SOLVER_DFSPH)
    wcsph = solver == scenes.SOLVER_WCSPH
    arms = ["plain", "learned"] if args.arm == "both" else [args.arm]
    if solver != scenes.SOLVER_DFSPH:
        arms = ["plain"]   # the learned warm start is DFSPH's
    if "learned" in arms and not os.path.exists(weights):
        print("[bench] no trained warm-start weights; learned arm skipped", flush=True)
        arms = [a for a in arms if a != "learned"] or ["plain"]
    results = {}
    for arm in arms:
        sim = sph.Simulation(sc, params=dict(sc.params, auto_rebuild=1))   # the step queues its own build
        net = None
        if arm == "learned":
            import numpy as np
            net = sph.MLP(np.fromfile(weights, dtype=np.float32))
            sim.set_warm_start(2, net)
        print(f"[bench] {sc.name} ({arm}): {sc.n_fluid} fluid, {sc.n_boundary} boundary, warmup {args.warmup}",
              flush=True)
        # the last few warmup steps time every kernel (the per-kernel table and
        # the choice of the dominant one); the timed steps then record the
        # events of the dominant kernel only, so that the throughput pays for
        # no other instrumentation
        # untimed steps past the start-up transient (the jitter's first
        # corrections, the first contact with the floor), so that the timed
        # window sees the flow the scene then keeps
        for _ in range(args.prerun):
            sim.advance()
        n_prof = min(5, args.warmup)
        for k in range(args.warmup):
            if k == args.warmup - n_prof:
                torch.cuda.synchronize()
                sim.profile_enable(True)
            sim.advance()
        torch.cuda.synchronize()
        prof_warm = {k: sim.profile_read(k) for k in PROFILED} if n_prof else {}
        dom = max(prof_warm, key=lambda k: prof_warm[k]["ms"]) if n_prof else None
        sim.profile_enable(True, only=dom)
        iters, walls = [], []
        for rep in range(max(1, args.reps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                st = sim.advance()
                iters.append((st["iters_div"], st["iters_dens"], st["cg_iters"], st["err_dens"], st["err_div"],
                              st["dt"]))
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        prof = {k: sim.profile_read(k) for k in PROFILED}
        sim.profile_enable(False)
        info = sim.info()
        sim.close()
        if net is not None:
            net.close()
        wall = sorted(walls)[len(walls) // 2]   # the median repetition
        print(f"[bench] {arm}: {len(walls)} x {args.steps} timed steps after {args.prerun} + {args.warmup}: "
              + ", ".join(f"{w:.4f}" for w in walls) + " s", flush=True)
        results[arm] = (wall, prof, iters, info, prof_warm if n_prof else prof, walls)
    wall, prof, iters, info, prof_table, walls = results[arms[0]]

    ms_step = wall * 1e3 / args.steps
    value = sc.n_fluid * args.steps / wall
    # dominant kernel: most event time (over the profiled warmup steps), its
    # launches timed over the timed region
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    achieved = (d["bytes"] / max(d["launches"], 1)) / (avg_ms * 1e-3) / 1e9 if d["launches"] else 0.0
    n_table = min(5, args.warmup) or args.steps
    table_ms = max(1e-9, sum(v["ms"] for v in prof_table.values()))
    kernels = {k: {"launches": v["launches"], "avg_us": (1e3 * v["ms"] / v["launches"]) if v["launches"] else 0.0,
                   "GBs": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else 0.0,
                   "share_of_kernel_time": v["ms"] / table_ms}
               for k, v in prof_table.items() if v["launches"]}
    n = len(iters)
    line = {
        "metric": ("particle-steps/sec (WCSPH, equation of state k=%g Pa, gamma=%g)"
                   % (sc.params["wcsph_k"], sc.params["wcsph_gamma"]) if wcsph else
                   "particle-steps/sec at eta=0.1% (PCISPH)" if solver == scenes.SOLVER_PCISPH else
                   "particle-steps/sec at eta=0.1% (DFSPH), plain vs learned warm start"),
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "prerun": args.prerun,
        "repetitions_s": walls,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "n_fluid": sc.n_fluid, "n_boundary": sc.n_boundary,
                   "n_rigid": len(sc.rigid), "r": sc.params["r"], "eta": sc.params["eta_density"],
                   "solver": ("dfsph", "wcsph", "pcisph")[solver], "dt_max": sc.params["dt_max"],
                   "warm_start": arms[0], "parallelism": "none (1 GPU)"},
        "iters_per_step": {"div": sum(i[0] for i in iters) / n, "dens": sum(i[1] for i in iters) / n,
                           "cg": sum(i[2] for i in iters) / n},
        "max_err_dens": max(i[3] for i in iters), "max_err_div": max(i[4] for i in iters),
        "mean_dt": sum(i[5] for i in iters) / n, "simulated_s_per_wall_s": sum(i[5] for i in iters) / wall,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.config, dom),
                     "bytes_per_launch": d["bytes"] / max(d["launches"], 1),
                     "launches": d["launches"], "avg_us": 1e3 * avg_ms},
        "kernels": kernels,
        "kernels_window": f"every kernel timed over the last {n_table} warmup steps",
    }
    if "learned" in results:
        lw, _, lit, _, lprof, lwalls = results["learned"]
        line["learned"] = {
            "value": sc.n_fluid * args.steps / lw, "ms_per_step": lw * 1e3 / args.steps, "repetitions_s": lwalls,
            "iters_per_step": {"div": sum(i[0] for i in lit) / len(lit), "dens": sum(i[1] for i in lit) / len(lit)},
            "max_err_dens": max(i[3] for i in lit),
            "warm_start_overhead_us": {k: (1e3 * lprof[k]["ms"] / max(1, lprof[k]["launches"]))
                                       for k in ("warm_features", "mlp") if lprof[k]["launches"]},
        }
        line["learned"]["speedup_vs_plain"] = line["learned"]["value"] / line["value"]
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", flush=True)
        line["cpu_baseline"] = cpu_baseline(args.config, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
