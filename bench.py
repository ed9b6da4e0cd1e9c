"""Benchmark: velocity updates per second of the MPM-2P operator splitting on one MI355X.

A step is one pass of the while loop of Algorithm 1 (Section 4.2): C_n upwind transport
sub-steps, kappa^n and epsilon, then a velocity update (MRCM with a new basis when
epsilon > eta, else MPM-2P with the stored one), downscaling and the next time step.
Workload: 1024^2 cells, 64x64 subdomains of 16^2 cells, 8 interface elements per side,
log-normal permeability with log-variance 4 (seeded, synthetic), viscosity ratio 100.
The initial MRCM (Algorithm 1, first lines) and the warm-up steps are outside the timed
region; inputs are resident in HBM before it starts.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(cfg: dict) -> dict:
    """Bytes each kernel class must move per launch at this workload (FP64 path).

    Cell fields are 8 B per cell, face fields 8 B per face. Per subdomain: the stored local
    factor nc (b+1) doubles, the Robin-to-flux map nb^2 doubles, boundary vectors nb doubles.
    """
    nx, ny, mx, my = cfg["nx"], cfg["ny"], cfg["sub_x"], cfg["sub_y"]
    nc = nx * ny
    nfaces = ny * (nx + 1) + (ny + 1) * nx
    nsub = (nx // mx) * (ny // my)
    b = min(mx, my)
    nb = 2 * (mx + my)
    ndof = 4 * (cfg["ne_x"] + cfg["ne_y"])
    return {
        # s, K, kappa^m read; kappa^n written
        "kappa_eps": 32.0 * nc,
        # s read, four face fluxes per cell (each face shared: ~2 faces per cell), s written
        "sat_step": 8.0 * nc + 8.0 * nfaces + 8.0 * nc,
        # factor read; kappa^n, kappa^m, q read; u~^m read; h, v written; interface rhs written
        "mpm_local": 8.0 * nsub * mx * my * (b + 1) + 24.0 * nc + 8.0 * nfaces + 16.0 * nsub * nb + 8.0 * nsub * ndof,
        # Robin-to-flux map, h, v read; boundary fluxes written
        "flux": 8.0 * nsub * nb * nb + 24.0 * nsub * nb,
        # kappa, q read; boundary fluxes read (own + neighbour); velocity written
        "downscale": 16.0 * nc + 16.0 * nsub * nb + 8.0 * nfaces,
    }


def roc_info():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        model = [l.split(":", 1)[1].strip() for l in out.splitlines() if l.startswith("Model name")]
        return model[0] if model else platform.processor()
    except Exception:
        return platform.processor()


def cpu_baseline(cfg: dict, K: np.ndarray, steps: int = 3) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the workload: the 256^2 corner
    window of the same permeability with the same subdomain size and interface elements,
    one initial MRCM update then `steps` MPM-2P steps timed; the rate is scaled by the cell
    ratio (256^2 / 1024^2) to the full grid."""
    from threadpoolctl import threadpool_limits

    from oracle import splitting
    w = 256
    sub = dict(cfg, nx=w, ny=w, lx=cfg["lx"] * w / cfg["nx"], ly=cfg["ly"] * w / cfg["ny"])
    Kw = np.ascontiguousarray(K[:w, :w])
    with threadpool_limits(1):
        run = splitting.start(sub, Kw, np.zeros_like(Kw))
        t0 = time.perf_counter()
        for _ in range(steps):
            splitting.step(run, "mpm")
        dt = time.perf_counter() - t0
    rate_window = steps / dt
    scale = (w * w) / (cfg["nx"] * cfg["ny"])
    return {"value": rate_window * scale, "unit": "velocity updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle MPM-2P steps on the {w}x{w} corner window of the 1024^2 field "
                      f"({steps} steps after one MRCM update, {dt:.1f} s, 1 thread), rate scaled by the "
                      f"cell ratio {scale:.4f}; host: {roc_info()}, {os.cpu_count()} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              f"sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2103_11050_amd import binding, inputs

    cfg = inputs.config(args.workload)
    K = inputs.permeability(cfg)
    s0 = inputs.initial_saturation(cfg)
    dev = torch.device("cuda:0")
    Kt = torch.from_numpy(K).to(dev)
    st = torch.from_numpy(s0).to(dev)
    run = binding.Run(cfg, Kt, st)
    run.start()
    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    s_before = run.stats()
    stream = run.stream
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        run.step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s_after = run.stats()
    elapsed = t1 - t0
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    n_mrcm = s_after["tm"] - s_before["tm"]
    value = args.steps / elapsed

    # kernel timing with HIP events on the run's stream (separate short window)
    run.profile(enable=True, reset=True)
    for _ in range(args.profile_steps):
        run.step()
    prof = run.profile(enable=False, reset=True)
    # latency of a basis update (MRCM), forced after the timed window
    torch.cuda.synchronize()
    mr = []
    run.profile(enable=True, reset=True)
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run.step(binding.FORCE_MRCM)
        e1.record(stream)
        torch.cuda.synchronize()
        mr.append(e0.elapsed_time(e1))
    mprof = run.profile(enable=False, reset=True)
    alg = algorithmic_bytes(cfg)
    cand = {k: v for k, v in prof.items() if k in alg}
    dom = max(cand, key=lambda k: cand[k][0]) if cand else None
    roof = None
    if dom:
        ms = cand[dom][0]
        achieved = alg[dom] / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_ms": round(ms, 5), "algorithmic_bytes": alg[dom]}
    out = {
        "metric": "velocity updates/s (MRCM + MPM-2P) at 1024^2 cells; p50/p99 run latency; %roofline",
        "value": round(value, 2),
        "unit": "velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1024^2 cells, 64x64 subdomains of 16^2, 8 interface elements per side, "
                               "log-normal K (log-variance 4, correlation length 0.05, seed 3), M=100, eta=0.1, C_n=1",
                   "mrcm_updates_in_window": int(n_mrcm), "mpm_steps_in_window": int(args.steps - n_mrcm),
                   "step_latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                   "step_latency_ms_p99": round(float(np.percentile(lat, 99)), 4)},
        "roofline": roof,
        "kernels_ms": {k: round(v[0], 5) for k, v in sorted(prof.items())},
        "mrcm_update_ms": round(float(np.median(mr)), 4),
        "mrcm_kernels_ms": {k: round(v[0], 5) for k, v in sorted(mprof.items())},
    }
    run.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, K)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
