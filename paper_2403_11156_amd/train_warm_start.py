"""Train the learned warm start of the density solve on the device.

1. Trace collection: run the plain solver (previous-step warm start) on the
   8k dam break (c1, all 100 steps) and the 125k dam break (c2, every 10th of
   1000 steps); each traced step appends, per fluid particle, the five
   features at the start of the density solve and the step's final stiffness
   (sph_enable_trace) into device tensors.
   With --dagger WEIGHTS the same runs are traced again with the learned
   start of those weights, and both sets of traces are trained on (the
   network then also sees the states its own trajectories reach).
2. Training: mean squared error of the normalised prediction, Adam on the
   device (sph_mlp_train_step: bf16 matrix-core forward and backward, FP32
   master weights), shuffled mini-batches.
3. The FP32 parameters go to weights/warm_start_mlp.f32 with a JSON record.

    python -m paper_2403_11156_amd.train_warm_start [--epochs 40] [--quick]
        [--runs c1:100:1,c2:1000:10] [--dagger WEIGHTS] [--out PATH]
"""

from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "warm_start_mlp.f32")
RECORD = os.path.join(HERE, "weights", "warm_start_mlp.json")
H = 64


def init_params(seed, shift, scale, out_scale):
    """He-uniform initial weights, normalisation folded into the layout."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (H, 5)) * np.sqrt(6.0 / 5), np.zeros(H),
             rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H), np.zeros(H),
             rng.uniform(-1, 1, H) * np.sqrt(6.0 / H) * 0.1, np.zeros(1),
             np.asarray(shift, np.float64), np.asarray(scale, np.float64), np.array([out_scale])]
    return np.concatenate([np.asarray(a, np.float64).reshape(-1) for a in parts]).astype(np.float32)


def collect(runs, torch, sph, scenes, log=print, net_params=None):
    """runs: list of (scene name, steps, trace every k-th step).  With
    net_params the runs take the learned start of that network, so the
    traces cover the states its own trajectories reach."""
    total = 0
    for name, steps, every in runs:
        total += scenes.scene(name).n_fluid * len(range(0, steps, every))
    F = torch.zeros((total, 5), dtype=torch.float32, device="cuda")
    T = torch.zeros(total, dtype=torch.float32, device="cuda")
    row = 0
    for name, steps, every in runs:
        sc = scenes.scene(name)
        sim = sph.Simulation(sc)
        net = None
        if net_params is not None:
            net = sph.MLP(net_params)
            sim.set_warm_start(2, net)
        t0 = time.time()
        iters = []
        for s in range(steps):
            traced = s % every == 0
            if traced:
                sim.enable_trace(F[row:], T[row:], sc.n_fluid)
            st = sim.advance()
            iters.append(st["iters_dens"])
            if traced:
                assert sim.trace_rows() == sc.n_fluid
                row += sc.n_fluid
                sim.enable_trace(None, None, 0)
        torch.cuda.synchronize()
        log(f"[trace] {sc.name}{' (learned start)' if net is not None else ''}: {steps} steps in "
            f"{time.time() - t0:.1f} s, mean density iterations {np.mean(iters):.2f}, rows so far {row}")
        sim.close()
        if net is not None:
            net.close()
    return F, T


def train(F, T, torch, sph, epochs=40, batch=65536, lr=2e-3, halve_every=10, seed=0, log=print):
    n = F.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    perm = torch.randperm(n, generator=g, device="cuda")
    n_val = max(1, n // 20)
    val, tr = perm[:n_val], perm[n_val:]
    Fv, Tv = F[val].contiguous(), T[val].contiguous()
    Ft, Tt = F[tr].contiguous(), T[tr].contiguous()
    shift = Ft.mean(0).cpu().numpy()
    scale = 1.0 / np.maximum(Ft.std(0).cpu().numpy(), 1e-12)
    out_scale = float(max(Tt.std().item(), 1e-12))
    p0 = init_params(seed + 1, shift, scale, out_scale)
    net = sph.MLP(p0)
    hist = []
    base, _ = net.grad(Fv, Tv)
    # loss of the plain warm start on the same samples, for reference:
    # K0 = warm_factor * K_prev is feature 3 times the warm factor
    log(f"[train] {Ft.shape[0]} training / {n_val} validation samples; initial validation loss {base:.4g}")
    steps_per_epoch = max(1, Ft.shape[0] // batch)
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        order = torch.randperm(Ft.shape[0], generator=g, device="cuda")
        rate = lr * (0.5 ** (ep // halve_every))
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            net.train_step(Ft[idx].contiguous(), Tt[idx].contiguous(), rate)
            step += 1
        v, _ = net.grad(Fv, Tv)
        hist.append(v)
        log(f"[train] epoch {ep + 1}/{epochs} lr {rate:.2e} validation loss {v:.4g} ({time.time() - t0:.1f} s)")
    params = net.params()
    net.close()
    return params, {"validation_loss": hist, "initial_validation_loss": base, "samples": int(n),
                    "train_steps": step, "batch": batch, "epochs": epochs, "lr": lr, "halve_every": halve_every}


def source_digest() -> str:
    """SHA-256 prefix of the sources the traces depend on (the HIP library and
    the scene generator), recorded with the weights."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(open(os.path.join(HERE, "scenes.py"), "rb").read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--quick", action="store_true", help="c1 only, 2 epochs (smoke of the driver)")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--dagger", default="",
                    help="weights whose learned start also runs the trace scenes; its traces join the plain ones")
    ap.add_argument("--runs", default="",
                    help="trace runs as name:steps:every,... (default c1:100:1,c2:1000:10)")
    ap.add_argument("--commit", default=os.environ.get("TRACE_COMMIT", ""),
                    help="the repository commit whose solver produced the traces (recorded)")
    args = ap.parse_args()
    import torch
    from paper_2403_11156_amd import scenes, sph
    torch.cuda.set_device(0)
    runs = [("c1", 100, 1)] if args.quick else [("c1", 100, 1), ("c2", 1000, 10)]
    if args.runs:
        runs = [(a, int(b), int(c)) for a, b, c in (r.split(":") for r in args.runs.split(","))]
    F, T = collect(runs, torch, sph, scenes)
    if args.dagger:
        dagger = np.fromfile(args.dagger, dtype=np.float32)
        F2, T2 = collect(runs, torch, sph, scenes, net_params=dagger)
        F, T = torch.cat([F, F2]), torch.cat([T, T2])
        del F2, T2
    params, rec = train(F, T, torch, sph, epochs=2 if args.quick else args.epochs)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    params.astype(np.float32).tofile(args.out)
    rec["runs"] = runs
    rec["trace_windows"] = [f"{name}: steps 0..{steps - 1}, every {every}" for name, steps, every in runs]
    rec["source_digest"] = source_digest()
    if args.dagger:
        import hashlib
        rec["dagger_from"] = hashlib.sha256(open(args.dagger, "rb").read()).hexdigest()[:16]
    rec["commit"] = args.commit
    keys = ("warm_start", "warm_factor", "alpha_max_factor", "eta_density", "eta_density_max", "eta_divergence",
            "cfl_lambda", "dt_max", "visc_model", "visc")
    rec["solver_readings"] = {name: {k: scenes.scene(name).params.get(k) for k in keys} for name, _, _ in runs}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"weights": args.out, **{k: rec[k] for k in ("samples", "train_steps")},
                      "final_validation_loss": rec["validation_loss"][-1]}))


if __name__ == "__main__":
    main()
