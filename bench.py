"""Benchmark: velocity updates per second of the MPM-2P operator splitting on one MI355X.

A step is one pass of the while loop of Algorithm 1 (Section 4.2): C_n upwind transport
sub-steps, kappa^n and epsilon, then a velocity update (MRCM with a new basis when
epsilon > eta, else MPM-2P with the stored one), downscaling and the next time step.
Workload: 1024^2 cells, 64x64 subdomains of 16^2 cells, 8 interface elements per side,
log-normal permeability with log-variance 4 (seeded, synthetic), viscosity ratio 100.
The initial MRCM (Algorithm 1, first lines) and the warm-up steps are outside the timed
region; inputs are resident in HBM before it starts.

Prints one JSON line. Extra modes: --copy-probe-mib (a plain device copy, to calibrate the
HBM counters) and --make-traffic (builds the traffic record from rocprofv3 counter output).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_1024.json")
# sources of the kernels each traffic record covers (the record is void once they change)
KERNEL_SOURCES = {
    "mpm_local": ["lines.hip", "lines.hpp", "device.hpp", "kernels.hpp"],
    "downscale": ["lines.hip", "lines.hpp", "device.hpp"],
    "flux": ["local.hip", "device.hpp"],
    "sat_kappa": ["local.hip", "device.hpp"],
    "sat_step": ["transport.hip", "device.hpp"],
    "iface_sub_fwd": ["nd.hip", "device.hpp", "kernels.hpp", "plan.hpp", "plan.cpp"],
    "iface_sub_bwd_flux": ["nd.hip", "device.hpp", "kernels.hpp", "plan.hpp", "plan.cpp"],
}
# rocprofv3 kernel names -> kernel classes of the library's event profiler (the fused backward
# sweep by its instance: with the reconstruction or without)
TRAFFIC_NAMES = {"k_mpm_local_lb": "mpm_local", "k_downscale_lb": "downscale", "k_flux": "flux",
                 "k_kappa": "sat_kappa", "k_sat_step": "sat_step", "k_nd_sub_fwd": "iface_sub_fwd",
                 "k_nd_sub_bwd<true>": "iface_sub_bwd_flux"}


def algorithmic_bytes(cfg: dict) -> dict:
    """Bytes each kernel class must move per launch at this workload (FP64 path).

    Cell fields are 8 B per cell, face fields 8 B per face. Per subdomain: the kept line-block
    inverses (symmetric, so lines x 16 (16 + 1) / 2 doubles of their upper triangles, lines
    padded to 8 or 16 cells), the symmetric Robin-to-flux map ((nb / 2 + 1) nb doubles of its
    wrapped diagonals), boundary vectors nb doubles (nb = 2 (mx + my)).
    """
    nx, ny, mx, my = cfg["nx"], cfg["ny"], cfg["sub_x"], cfg["sub_y"]
    nc = nx * ny
    nfaces = ny * (nx + 1) + (ny + 1) * nx
    nsub = (nx // mx) * (ny // my)
    band = min(mx, my)
    mf = 8 if band <= 8 else 16 if band <= 16 else 32
    blocks = 8.0 * nsub * (mx * my // band) * (mf * (mf + 1) // 2)
    nb = 2 * (mx + my)
    ndof = 4 * (cfg["ne_x"] + cfg["ne_y"])
    return {
        # last transport sub-step with the conductivity: s, four face fluxes per cell (each
        # face shared), K, kappa^m read; s and kappa^n written
        "sat_kappa": 8.0 * nc + 8.0 * nfaces + 8.0 * nc + 24.0 * nc,
        # the other C_n - 1 sub-steps: s and the faces read, s written
        "sat_step": 8.0 * nc + 8.0 * nfaces + 8.0 * nc,
        # kept blocks; kappa^n, kappa^m, q; u~^m; h and v written; interface rhs written
        "mpm_local": blocks + 24.0 * nc + 8.0 * nfaces + 16.0 * nsub * nb + 8.0 * nsub * ndof,
        # Robin-to-flux map (symmetric: nb / 2 + 1 wrapped diagonals), h, v read; fluxes written
        "flux": 8.0 * nsub * (nb // 2 + 1) * nb + 24.0 * nsub * nb,
        # kept blocks; kappa, q; boundary fluxes (own + neighbour); velocity written
        "downscale": blocks + 16.0 * nc + 16.0 * nsub * nb + 8.0 * nfaces,
    }


def phase_rooflines(alg: dict, sb: dict, prof: dict, cfg: dict, ms_step: float) -> dict:
    """HBM rooflines of the interface sweeps (many level kernels each, so not a single-kernel
    figure) and of the whole MPM-2P step (sum of the algorithmic bytes of its kernels; the
    Neumann refactorisation of changed subdomains and the scalar reductions left out). Where the
    backward sweep also reconstructs the boundary fluxes (no flux phase of its own), its bytes
    include the reconstruction's."""
    out = {}
    fused_flux = "flux" not in prof
    for name, key in (("iface_fwd", "fwd"), ("iface_bwd", "bwd")):
        if name in prof and prof[name][0] > 0:
            nbytes = sb[key] + (alg["flux"] if key == "bwd" and fused_flux else 0.0)
            gbs = nbytes / (prof[name][0] * 1e-3) / 1e9
            out[name] = {"bytes": nbytes, "ms": round(prof[name][0], 5), "achieved": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
            if key == "bwd" and fused_flux:
                out[name]["note"] = "with the reconstruction of the boundary fluxes"
    step_bytes = sum(alg[k] * (cfg["cn"] - 1 if k == "sat_step" else 1) for k in alg) + sb["fwd"] + sb["bwd"]
    gbs = step_bytes / (ms_step * 1e-3) / 1e9
    out["step"] = {"bytes": step_bytes, "ms": round(ms_step, 4), "achieved": round(gbs, 1),
                   "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_2103_11050_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter record, if it was taken on
    the current source of that kernel; None otherwise."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_hash") != source_hash(kernel):
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def _per_kernel(path):
    """Counter values per kernel (FP64 instances only: the FP32-block instances of the
    precision form are left out)."""
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        full = r["Kernel_Name"].split("(")[0]
        if "float" in full:
            continue
        name = full.split("<")[0].replace("void ", "").replace("mpm::", "")
        if name == "k_nd_sub_bwd":
            name = full.replace("void ", "").replace("mpm::", "").strip()
        d[name].append(float(r["Counter_Value"]))
    return d


def make_traffic(fetch, write, cfetch, cwrite):
    """Writes the traffic record from two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE) and the same counters on a plain device copy (--copy-probe-mib 256), which
    calibrates KiB-per-dispatch to bytes."""
    f, w = _per_kernel(fetch), _per_kernel(write)
    cf, cw = _per_kernel(cfetch), _per_kernel(cwrite)
    copy_bytes = 256 * (1 << 20)
    kf = copy_bytes / (1024.0 * max(cf["__amd_rocclr_copyBuffer"]))
    kw = copy_bytes / (1024.0 * max(cw["__amd_rocclr_copyBuffer"]))
    out = {"calibration": {"copy_bytes": copy_bytes, "fetch_scale": kf, "write_scale": kw,
                           "note": "bytes = counter KiB * 1024 * scale; scale from a plain copy"},
           "kernels": {}}
    for raw, name in TRAFFIC_NAMES.items():
        if raw not in f:
            continue
        # median over the dispatches: the MPM-2P steps outnumber the MRCM updates in the
        # profiled run (the downscaling of an MRCM update also writes the kept factors)
        fv, wv = f[raw], w.get(raw, [0.0])
        out["kernels"][name] = {
            "fetch_bytes": float(np.median(fv)) * 1024 * kf, "write_bytes": float(np.median(wv)) * 1024 * kw,
            "dispatches": len(fv), "source_hash": source_hash(name)}
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out, indent=1))


def host_cpu():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        model = [l.split(":", 1)[1].strip() for l in out.splitlines() if l.startswith("Model name")]
        return model[0] if model else platform.processor()
    except Exception:
        return platform.processor()


def cpu_baseline(cfg: dict, K: np.ndarray, steps: int = 40) -> dict:
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
                      f"cell ratio {scale:.4f}; host: {host_cpu()}, {os.cpu_count()} logical CPUs"}


def precision_form(binding, cfg, Kt, st, steps: int, warmup: int, rtols=(1e-6, 1e-10)) -> dict:
    """The precision form (FP32 inverse blocks in the MPM-2P local solves and downscaling, FP64
    refinement to refine_rtol, FP64 interface solve and switch criterion) beside the FP64 path on
    the same workload: its rate over `steps` steps and its velocity difference from the FP64
    path after the same steps from the same start, for each refinement target (the first is the
    headline one)."""
    import torch

    def timed(c, prec):
        r = binding.Run(c, Kt, st, precision=prec)
        r.start()
        for _ in range(warmup):
            r.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r.step()
        torch.cuda.synchronize()
        return r, steps / (time.perf_counter() - t0)

    def rt0(ux, uy):   # velocity norm of the lowest-order mixed space with the trapezoidal rule
        return np.sum(ux[:, :-1] ** 2) + np.sum(ux[:, 1:] ** 2) + np.sum(uy[:-1, :] ** 2) + np.sum(uy[1:, :] ** 2)

    r64, v64 = timed(cfg, binding.PREC_FP64)
    ux64, uy64 = (t.cpu().numpy() for t in r64.velocity())
    b64 = r64.stats()["last_branch"]
    r64.close()
    by = {}
    for rt in rtols:
        r32, v32 = timed(dict(cfg, refine_rtol=rt), binding.PREC_FP32_REFINE)
        ux32, uy32 = (t.cpu().numpy() for t in r32.velocity())
        s32 = r32.stats()
        r32.close()
        by[f"{rt:g}"] = {"value": round(v32, 2), "vel_rel_l2_vs_fp64": float(np.sqrt(rt0(ux32 - ux64, uy32 - uy64) /
                                                                                    rt0(ux64, uy64))),
                         "same_branches": bool(s32["last_branch"] == b64), "error_word": int(s32["error_word"])}
    head = by[f"{rtols[0]:g}"]
    return {"value": head["value"], "refine_rtol": rtols[0], "fp64_value_same_window": round(v64, 2),
            "steps": steps, "vel_rel_l2_vs_fp64": head["vel_rel_l2_vs_fp64"], "same_branches": head["same_branches"],
            "by_refine_rtol": by,
            "note": "FP32 blocks applied in FP32, FP64 iterative refinement of every local solve to refine_rtol"}


def _side_by_side(binding, cfg, Kt, st, steps: int, warmup: int, over: dict):
    """Rates of the workload as given and with the descriptor fields `over` changed, over the
    same window, and the relative RT0 difference of the two velocities after it."""
    import torch

    runs = []
    for c in (cfg, dict(cfg, **over)):
        r = binding.Run(c, Kt, st)
        r.start()
        for _ in range(warmup):
            r.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r.step()
        torch.cuda.synchronize()
        runs.append((r, steps / (time.perf_counter() - t0)))
    (r0, v0), (r1, v1) = runs
    ux0, uy0 = (t.cpu().numpy() for t in r0.velocity())
    ux1, uy1 = (t.cpu().numpy() for t in r1.velocity())

    def rt0(ux, uy):
        return np.sum(ux[:, :-1] ** 2) + np.sum(ux[:, 1:] ** 2) + np.sum(uy[:-1, :] ** 2) + np.sum(uy[1:, :] ** 2)

    diff = float(np.sqrt(rt0(ux1 - ux0, uy1 - uy0) / rt0(ux0, uy0)))
    s0, s1 = r0.stats(), r1.stats()
    upd = []
    for r in (r0, r1):   # median time of a forced MRCM update (basis, interface factorisation)
        t = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.step(binding.FORCE_MRCM)
            torch.cuda.synchronize()
            t.append(1e3 * (time.perf_counter() - t0))
        upd.append(round(float(np.median(t)), 3))
    r0.close()
    r1.close()
    return v0, v1, diff, s0, s1, upd


def first_order_form(binding, cfg, Kt, st, steps: int, warmup: int) -> dict:
    """MPM-2P with the first-order term of eq:mpm_tf_4 (mpm_order = 1) beside the zeroth-order
    path on the same workload: its rate over `steps` steps and the relative difference of the two
    velocities after them (the size of the term the paper neglects)."""
    v0, v1, diff, s0, s1, _ = _side_by_side(binding, cfg, Kt, st, steps, warmup, {"mpm_order": 1})
    return {"value": round(v1, 2), "zeroth_order_value_same_window": round(v0, 2), "steps": steps,
            "vel_rel_l2_first_minus_zeroth": diff, "same_basis_count": s0["tm"] == s1["tm"],
            "note": "one more local solve per subdomain, interface solve and reconstruction per step"}


def linear_space_form(binding, cfg, Kt, st, steps: int, warmup: int) -> dict:
    """The same workload with the -POL interface spaces of Section 5.2 (iface_degree = 1: U_H,
    P_H linear per element, twice the interface unknowns): its rate and the relative difference
    of its velocity from the piecewise-constant one after the window."""
    v0, v1, diff, s0, s1, upd = _side_by_side(binding, cfg, Kt, st, steps, warmup, {"iface_degree": 1})
    return {"value": round(v1, 2), "constant_space_value_same_window": round(v0, 2), "steps": steps,
            "vel_rel_l2_linear_minus_constant": diff, "basis_updates": [s0["tm"], s1["tm"]],
            "mrcm_update_ms_constant_linear": upd,
            "note": "k_U = k_P = 2 per interface element; the interface system has twice the unknowns"}


def serving_form(binding, inputs, n_requests: int, refine_rtol: float) -> dict:
    """The serving form on a short request stream: grids drawn from 128^2, 256^2, 512^2 (16^2
    subdomains, 4 elements per side), log-variance in [1, 4], M in [10, 100], each request run to
    breakthrough, 16 slots. FP64: the capacity (all requests at t = 0), then Poisson arrivals at
    70 % of it with p50/p99 latency. The precision form (FP32 blocks refined to refine_rtol) on the
    same requests, capacity and the same arrival stream; its accuracy is the relative RT0
    difference of each request's final velocity from the FP64 one (largest over the requests)."""
    from paper_2103_11050_amd import serve

    reqs = inputs.serve_requests(n_requests, (128, 256, 512))
    reqs32 = [dict(c, refine_rtol=refine_rtol) for c in reqs]
    budget = 200 << 30
    s64, s32 = [], []
    f64 = serve.serve_measure(reqs, 16, budget, 100000, 0.0, binding.PREC_FP64, states=s64)
    f32 = serve.serve_measure(reqs32, 16, budget, 100000, f64["rate_per_s"], binding.PREC_FP32_REFINE,
                              measure_capacity=True, states=s32)

    def rt0(ux, uy):
        return np.sum(ux[:, :-1] ** 2) + np.sum(ux[:, 1:] ** 2) + np.sum(uy[:-1, :] ** 2) + np.sum(uy[1:, :] ** 2)

    diffs = [float(np.sqrt(rt0(a[0] - b[0], a[1] - b[1]) / rt0(a[0], a[1]))) for a, b in zip(s64, s32)]
    same = sum(1 for a, b in zip(s64, s32) if a[3] == b[3])
    keys = ("runs_per_s", "velocity_updates_per_s", "latency_p50_s", "latency_p99_s", "mean_runs_per_batch_step")
    return {"requests": n_requests, "rate_per_s": f64["rate_per_s"],
            "fp64": {**{k: f64[k] for k in keys}, "capacity": f64["capacity_measured"]},
            "precision_form": {**{k: f32[k] for k in keys}, "capacity": f32["capacity_measured"],
                               "refine_rtol": refine_rtol, "vel_rel_l2_vs_fp64_max": max(diffs),
                               "requests_same_pass_count": same},
            "note": "latency from arrival to breakthrough; capacity with every request present at t = 0; "
                    "requests' fields made before the first arrival"}


def long_window(binding, cfg, Kt, st, updates: int) -> dict:
    """Algorithm 1 over a long window from s = 0 (MRCM updates wherever the switch asks for
    them): the whole-job rate with the basis updates inside the timed region."""
    import torch

    r = binding.Run(cfg, Kt, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r.start()
    done = 0
    while done < updates:
        k = r.advance(min(500, updates - done))
        done += k
        if k == 0 or r.stats()["breakthrough"]:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s = r.stats()
    r.close()
    return {"velocity_updates": int(s["te"]), "basis_sets": int(s["tm"]), "seconds": round(el, 4),
            "updates_per_s": round(s["te"] / el, 2), "pvi": round(float(s["pvi"]), 5),
            "note": "start (initial basis) and every update of the window timed, MRCM updates included"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", choices=["fp64", "fp32-refine"], default="fp64",
                    help="local solves with FP64 blocks, or FP32 blocks with FP64 refinement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-form", action="store_true",  # also skips the other side forms
                    help="skip the side-by-side run of the FP32-block precision form")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--tune", type=int, default=1, help="autotune the interface-sweep launch shapes (1) or "
                    "keep the fixed rule (0)")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests of the served-form figures (p50/p99 run latency; 0: skip)")
    ap.add_argument("--refine-rtol", type=float, default=1e-6,
                    help="refinement target of the precision form (its velocity bound is 1e-6)")
    ap.add_argument("--long-window", type=int, default=6000,
                    help="velocity updates of the long-window figure (0: skip)")
    ap.add_argument("--make-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="build the traffic record from rocprofv3 --pmc outputs and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.make_traffic:
        make_traffic(*args.make_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU "
              f"sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 8 * n, "launches": 5}))
        return

    from paper_2103_11050_amd import binding, inputs

    cfg = inputs.config(args.workload)
    K = inputs.permeability(cfg)
    s0 = inputs.initial_saturation(cfg)
    dev = torch.device("cuda:0")
    Kt = torch.from_numpy(K).to(dev)
    st = torch.from_numpy(s0).to(dev)
    prec = binding.PREC_FP64 if args.precision == "fp64" else binding.PREC_FP32_REFINE
    run = binding.Run(cfg, Kt, st, precision=prec)
    run.start()
    # interface-sweep launch shapes: autotuned once per decomposition (also used by every later
    # run of this decomposition in the process)
    tuned = run.tune(5) if args.tune else None
    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    s_before = run.stats()
    stream = run.stream
    # throughput window: nothing but the steps between the two synchronisations
    t0 = time.perf_counter()
    for k in range(args.steps):
        run.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s_after = run.stats()
    elapsed = t1 - t0
    n_mrcm = s_after["tm"] - s_before["tm"]
    value = args.steps / elapsed
    # per-step latency window (an event per step, which itself costs a few microseconds)
    nlat = min(args.steps, 100)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nlat + 1)]
    evs[0].record(stream)
    for k in range(nlat):
        run.step()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(nlat)])

    # kernel timing with HIP events on the run's stream (separate short window)
    run.profile(enable=True, reset=True)
    for _ in range(args.profile_steps):
        run.step()
    prof = run.profile(enable=False, reset=True)
    # the fused sweep launches timed in a window of their own (their events would add to the
    # phases above)
    run.profile(enable=2, reset=True)
    for _ in range(args.profile_steps):
        run.step()
    fine = run.profile(enable=False, reset=True)
    for k in ("iface_sub_fwd", "iface_sub_bwd_flux", "iface_sub_bwd"):
        if k in fine:
            prof[k] = fine[k]
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
    sb = run.solve_bytes()
    # single launches with their algorithmic bytes: the per-subdomain kernels, and the fused
    # bottom levels of the interface sweeps (the backward one with the reconstruction)
    fb = run.fused_bytes()
    kern = dict(alg)
    if fb["levels"] > 0:
        kern["iface_sub_fwd"] = float(fb["fwd"])
        kern["iface_sub_bwd_flux"] = float(fb["bwd"]) + alg["flux"]
        kern["iface_sub_bwd"] = float(fb["bwd"])
    cand = {k: v for k, v in prof.items() if k in kern}
    dom = max(cand, key=lambda k: cand[k][0]) if cand else None
    roof = None
    if dom:
        ms = cand[dom][0]
        achieved = kern[dom] / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                "avg_ms": round(ms, 5), "algorithmic_bytes": kern[dom]}
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
        "dtype": "f64" if args.precision == "fp64" else "f32 blocks + f64 refinement (interface, residuals, epsilon f64)",
        "data": "synthetic",
        "config": {"workload": "1024^2 cells, 64x64 subdomains of 16^2, 8 interface elements per side, "
                               "log-normal K (log-variance 4, correlation length 0.05, seed 3), M=100, eta=0.1, C_n=1",
                   "mrcm_updates_in_window": int(n_mrcm), "mpm_steps_in_window": int(args.steps - n_mrcm),
                   "step_latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                   "step_latency_ms_p99": round(float(np.percentile(lat, 99)), 4)},
        "roofline": roof,
        "phases": phase_rooflines(alg, sb, prof, cfg, 1e3 * elapsed / args.steps),
        "kernels_ms": {k: round(v[0], 5) for k, v in sorted(prof.items())},
        "mrcm_update_ms": round(float(np.median(mr)), 4),
        "sweep_tuning": None if tuned is None else {
            "solve_ms_rule": round(tuned["ms_rule"], 4), "solve_ms_tuned": round(tuned["ms_tuned"], 4),
            "shapes": [list(x) for x in tuned["shapes"]],
            "note": "lanes per row, 16-byte column pairs per lane, rows per lane group of each sweep launch "
                    "(forward levels upwards, then backward levels downwards)"},
        "mrcm_kernels_ms": {k: round(v[0], 5) for k, v in sorted(mprof.items())},
    }
    run.close()
    if args.precision == "fp64" and not args.no_precision_form:
        out["precision_form"] = precision_form(binding, cfg, Kt, st, min(args.steps, 100), args.warmup,
                                               (args.refine_rtol, 1e-10))
    if args.precision == "fp64" and not args.no_precision_form:
        out["first_order_form"] = first_order_form(binding, cfg, Kt, st, min(args.steps, 100), args.warmup)
        out["linear_space_form"] = linear_space_form(binding, cfg, Kt, st, min(args.steps, 100), args.warmup)
    if args.long_window > 0 and args.precision == "fp64":
        out["long_window"] = long_window(binding, cfg, Kt, st, args.long_window)
    if args.serve_requests > 0:
        out["serving"] = serving_form(binding, inputs, args.serve_requests, args.refine_rtol)
        out["config"]["run_latency_s_p50"] = out["serving"]["fp64"]["latency_p50_s"]
        out["config"]["run_latency_s_p99"] = out["serving"]["fp64"]["latency_p99_s"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, K)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
