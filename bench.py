#!/usr/bin/env python3
"""Benchmark of the local ETKF frame on one MI355X.

Workload: 80x80 Shack-Hartmann subapertures, 28 % central obscuration (4632
valid subapertures, 9264 slopes, 4836 valid actuator nodes), ensemble m = 64,
4x4-subaperture domains with a 1-subaperture halo (332 local analyses per
frame).  FP32 state and matrix-core contractions, FP64 eigensolve.  Synthetic
inputs: an AR(1) von Karman true phase, its Fried slopes plus N(0, 0.1^2)
noise, and model noise drawn on the device from a bank of von Karman screens.
All inputs are resident in HBM before timing starts.

One step = one letkf_step: the fused forecast, all local analyses in one
launch, the gather and the least-squares differential-piston removal (graph
replay).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LETKF frames/sec and local analyses/sec at 80×80 SH, m=64; batched vs plain"
COPY_BYTES = 256 << 20       # calibration copy of the profile run (read and written once)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_analysis_80x80_m64_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1408_7069_amd", "csrc", "letkf_kernels.hip")


def kernel_hash() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per analysis launch from the committed counter summary, or None
    when the kernel source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha256_16") != kernel_hash():
        return None
    return float(kv["hbm_bytes_per_launch"])
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (and matrix) peak
FP32_MFMA_PEAK_TFLOPS = 157.3
TRACE_FILE = os.path.join(ROOT, "profiles", "k_analysis_80x80_m64_trace.md")


def algorithmic_flops(m: int, p_list, n_list) -> dict:
    """Nominal work of one instance's analyses per frame.  Counted against the
    roofline: the symmetric EVD with vectors, 9 m^3 per domain (FP64), the Gram
    2 m^2 p_l and the update 2 n_l m^2 (FP32 matrix cores).  Reported beside it,
    not counted: the transform W = Q Gamma^{-1/2} Q^T (2 m^3), the mean update
    2 n_l m and the slope stencil with Y^T d (6 p_l m)."""
    p = np.asarray(p_list, dtype=np.float64)
    n = np.asarray(n_list, dtype=np.float64)
    d = len(p)
    return {"evd_fp64": 9.0 * m ** 3 * d, "gram_fp32": float(np.sum(2 * m * m * p)),
            "update_fp32": float(np.sum(2 * n * m * m)),
            "not_counted": {"transform_2m3": 2.0 * m ** 3 * d, "mean_update": float(np.sum(2 * n * m)),
                            "stencil_and_ytd": float(np.sum(6 * p * m))}}


def bound_seconds(fl: dict) -> float:
    """Lower-bound time of the counted work at the MI355X peaks: the FP64 part
    at 78.6 TFLOP/s, the FP32 matrix-core part at 157.3 TFLOP/s."""
    return (fl["evd_fp64"] / (FP64_PEAK_TFLOPS * 1e12)
            + (fl["gram_fp32"] + fl["update_fp32"]) / (FP32_MFMA_PEAK_TFLOPS * 1e12))


def handle_bound(f) -> tuple[float, dict]:
    """Sum of the per-instance lower bounds of a handle (each instance with its
    own m, p_l and n_l), and the summed counts."""
    t, tot = 0.0, {"evd_fp64": 0.0, "gram_fp32": 0.0, "update_fp32": 0.0}
    for i, sp in enumerate(f.specs):
        g = f.geometry(i)
        fl = algorithmic_flops(sp.m, np.diff(g["obs_off"]), np.diff(g["own_off"]))
        t += bound_seconds(fl)
        for k in tot:
            tot[k] += fl[k]
    return t, tot


def trace_kernel_ms():
    """Average k_analysis duration of the committed rocprofv3 trace when it was
    taken on the current kernel source, else None."""
    if not os.path.exists(TRACE_FILE):
        return None
    txt = open(TRACE_FILE).read()
    if f"kernel_sha256_16: {kernel_hash()}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("trace_kernel_avg_us:"):
            return float(line.split(":", 1)[1]) * 1e-3
    return None


def transform_name(B, t: int) -> str:
    for name, attr in TRANSFORMS.items():
        if getattr(B, attr) == t:
            return name.upper()
    return str(t)


def schedule_label(sched) -> str:
    g, order = sched
    orders = {0: "row-major item order", 1: "XCD-contiguous item order",
              2: "XCD-contiguous item order, cost-paired second dispatch round"}
    return ("graph-replayed" if g else "directly launched") + ", " + orders.get(int(order), f"order {order}")


def batched_line(B, spec, y, K, W, copies: int) -> dict:
    """`copies` instances of the workload in one launch: frame time (graph
    replay), the analysis kernel's duration (HIP events around its direct
    launches) and the roofline fraction of both, sum(T_lb) over the instances
    divided by that time."""
    import torch
    f = B.Letkf([spec] * copies)
    yc = y.repeat(1, copies) if copies > 1 else y
    f.set_schedule(True, 1)
    ms = time_steps(f, yc, K, W)
    f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    f.set_frame(0)
    f.set_schedule(False, 1)
    time_steps(f, yc, 0, W)
    f.set_timing(True)
    time_steps(f, yc, K, 0, offset=W)
    kt = float(np.mean(f.analysis_times()))
    f.set_timing(False)
    t_lb, _ = handle_bound(f)
    nd = int(f.sizes["n_domains"])
    f.close()
    return {"instances": copies, "domains": nd, "ms_per_step": round(ms, 4), "kernel_ms": round(kt, 4),
            "local_analyses_per_s": round(nd * 1000.0 / ms, 1),
            "t_lb_us": round(t_lb * 1e6, 3), "frac_kernel": round(t_lb / (kt * 1e-3), 4),
            "frac_frame": round(t_lb / (ms * 1e-3), 4)}


def paper_shape_lines(B, w, bank, seed, y, K, W, copies=(1, 4)) -> list:
    """The shape of the paper's timings (Sec. 5.3, Tables 1-2): m = 101, 4x4
    domains with a halo of 2 (9x9-node patches, up to 128 local slopes) on the
    80x80 pupil, FP32 state, pistons, bank noise -- the wide analysis kernel
    (8 wavefronts a domain, FP64 P-form iteration); `copies` instances in one
    launch.  Frame time by the tuned schedule, the kernel's own duration by
    HIP events around its direct launches, the roofline fraction on the same
    count as the headline (9 m^3 + Gram + update per domain, m = 101)."""
    import torch
    out = []
    for nc in copies:
        spec = B.InstanceSpec(n_sub=w.n_sub, m=101, domain_size=4, halo=2, obscuration=w.obscuration,
                              rho=w.rho, r_sigma2=w.sigma ** 2, ar_coeff=w.a, noise_bank=bank, seed=seed,
                              precision=B.FP32, piston=True)
        f = B.Letkf([spec] * nc)
        yc = y.repeat(1, nc) if nc > 1 else y
        sched = f.autotune(yc[0], frames=20)
        zero = lambda: (f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32,
                                                   device="cuda")), f.set_frame(0))
        zero()
        ms = time_steps(f, yc, K, W)
        zero()
        f.set_schedule(False, sched[1])
        time_steps(f, yc, 0, W)
        f.set_timing(True)
        time_steps(f, yc, K, 0, offset=W)
        kt = float(np.mean(f.analysis_times()))
        f.set_timing(False)
        t_lb, _ = handle_bound(f)
        nd = int(f.sizes["n_domains"])
        steps = (f.status()[1] >> 8) & 255
        out.append({"instances": nc, "domains": nd, "m": 101, "max_local_slopes": int(f.sizes["max_obs"]),
                    "max_patch_nodes": int(f.sizes["max_patch"]), "schedule": schedule_label(sched),
                    "ms_per_step": round(ms, 4), "frames_per_s": round(1000.0 / ms, 2),
                    "kernel_ms": round(kt, 4), "local_analyses_per_s": round(nd * 1000.0 / ms, 1),
                    "us_per_local_analysis_kernel": round(kt * 1000.0 / nd, 4),
                    "t_lb_us": round(t_lb * 1e6, 3), "frac_kernel": round(t_lb / (kt * 1e-3), 4),
                    "frac_frame": round(t_lb / (ms * 1e-3), 4),
                    "transform_steps_mean": round(float(steps.mean()), 3),
                    "paper_cpu_ms_per_domain": 0.94})
        f.close()
    return out


TRANSFORMS = {"nsp_mixed": "TRANSFORM_NSP_MIXED", "nsp": "TRANSFORM_NSP", "ns64": "TRANSFORM_NS64",
              "ns32": "TRANSFORM_NS32", "evd": "TRANSFORM_EVD"}
TRANSFORM_LABELS = {"nsp_mixed": "P-form Newton-Schulz, FP64 then FP32 steps",
                    "nsp": "P-form Newton-Schulz, FP64", "ns64": "coupled Newton-Schulz, FP64",
                    "ns32": "coupled Newton-Schulz, FP32 iterates", "evd": "Jacobi eigendecomposition, FP64"}


def transform_variants(B, spec, y, K, W, skip):
    """The same frames with the other transforms of the local analyses (frame
    time by graph replay, analysis kernel by HIP events)."""
    import dataclasses
    import torch
    out = {}
    for name, attr in TRANSFORMS.items():
        if name == skip:
            continue
        tr = getattr(B, attr)
        g = B.Letkf([dataclasses.replace(spec, transform=tr)])
        g.set_schedule(True, True)
        ms = time_steps(g, y, K, W)
        g.set_ensemble(torch.zeros(g.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
        g.set_frame(0)
        g.set_schedule(False, True)
        time_steps(g, y, 0, W)
        g.set_timing(True)
        time_steps(g, y, K, 0, offset=W)
        kt = float(np.mean(g.analysis_times()))
        g.set_timing(False)
        steps = (g.status()[1] >> 8) & 255
        out[name] = {"transform": TRANSFORM_LABELS[name], "ms_per_step": round(ms, 5),
                     "frames_per_s": round(1000.0 / ms, 2),
                     "kernel_ms": round(kt, 4), "steps_mean": round(float(steps.mean()), 3)}
        g.close()
    return out


def closed_loop_line(B, spec, wl_mod, w, y, truth, ij, K, W, frames=200):
    """The closed AO loop (Sec. 2.2 state: slopes of phi_{k-1} under the
    command u_{k-2}, command u_k from the analysis) on the same workload: frame
    time by graph replay on the staged slopes, then a loop of `frames` frames
    on the GPU with the sensor reading D (phi_{k-1} - u_{k-2}) + noise, and the
    variance of the residual phase phi_k - u_{k-1} over its second half."""
    import dataclasses
    import torch
    g = B.Letkf([dataclasses.replace(spec, model=B.MODEL_CLOSED_LOOP)])
    g.set_schedule(True, True)
    ms = time_steps(g, y, K, W)
    g.set_ensemble(torch.zeros(g.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    g.set_frame(0)
    n = g.sizes["n_nodes"]
    zero = torch.zeros(n, dtype=torch.float32, device="cuda")
    g.set_command(zero, zero)
    T = min(frames, truth.shape[0] - 1)
    ph = torch.from_numpy(np.ascontiguousarray(truth[:T + 1, ij[:, 0], ij[:, 1]], dtype=np.float32)).cuda()
    nrng = np.random.default_rng(w.seed + 2)
    noise = torch.from_numpy(wl_mod.gaussian_noise((T, g.sizes["n_slopes"]), w.sigma, nrng)
                             .astype(np.float32)).cuda()
    u1, u2 = zero.clone(), zero.clone()
    res, tur = [], []
    for k in range(1, T + 1):
        yk = g.slopes(ph[k - 1] - u2) + noise[k - 1]
        g.step(yk)
        if k > T // 2:
            r = ph[k] - u1
            res.append(float(torch.var(r, unbiased=False)))
            tur.append(float(torch.var(ph[k], unbiased=False)))
        u2, u1 = u1, g.get_command()
    g.close()
    return {"ms_per_step": round(ms, 5), "frames_per_s": round(1000.0 / ms, 2), "loop_frames": T,
            "residual_variance": round(float(np.mean(res)), 5), "phase_variance": round(float(np.mean(tur)), 3)}


def model_variants(B, spec, wl_mod, w, y, truth, ij, K, W, frames=300, a0s=(0.9, 0.9995), forgetting=0.98):
    """The turbulence-model variants on the same workload: frame times (graph
    replay) of the AR(2) forecast (a1 = 1.24, a2 = -0.26: lag correlations
    near 0.99 and 0.97) and of the online AR(1) refit, and for each
    mismatched a0 a loop over the staged slopes (true a = w.a) with model
    noise drawn for a0: the residual variance of the analysis mean over the
    second half with the model fixed at a0 and with the refit, and the
    refit's final coefficient; then the blend-mode gather: its frame time and
    the same residual variance against the concatenation with the piston
    step; covariance localisation likewise against the local analysis."""
    import dataclasses
    import torch
    out = {}
    g = B.Letkf([dataclasses.replace(spec, ar_coeff=1.24, ar2_coeff=-0.26)])
    g.set_schedule(True, True)
    out["ar2_ms_per_step"] = round(time_steps(g, y, K, W), 5)
    g.close()
    g = B.Letkf([dataclasses.replace(spec, refit_forgetting=forgetting)])
    g.set_schedule(True, True)
    out["refit_ms_per_step"] = round(time_steps(g, y, K, W), 5)
    g.close()
    T = min(frames, y.shape[0])
    ph = torch.from_numpy(np.ascontiguousarray(truth[:T, ij[:, 0], ij[:, 1]], dtype=np.float32)).cuda()
    loops = []
    for a0 in a0s:
        bank = wl_mod.bank_for(dataclasses.replace(w, a=a0), np.random.default_rng(w.seed + 3), n_screens=16)
        row = {"a0": a0}
        for name, fg in (("fixed", 0.0), ("refit", forgetting)):
            g = B.Letkf([dataclasses.replace(spec, ar_coeff=a0, noise_bank=bank, refit_forgetting=fg)])
            g.set_schedule(True, True)
            var = []
            for k in range(T):
                g.step(y[k])
                if k >= T // 2:
                    var.append(float(torch.var(g.get_mean() - ph[k], unbiased=False)))
            row[name + "_residual_variance"] = round(float(np.mean(var)), 5)
            if fg:
                row["refit_final_a"] = round(float(g.get_model()[0][0]), 5)
            g.close()
        loops.append(row)
    out.update({"true_a": w.a, "forgetting": forgetting, "loop_frames": T, "loops": loops})
    # the blend-mode gather against the concatenation with the piston step
    g = B.Letkf([dataclasses.replace(spec, gather_mode=B.GATHER_BLEND, piston=False)])
    g.set_schedule(True, True)
    blend = {"ms_per_step": round(time_steps(g, y, K, W), 5)}
    g.close()
    for name, kw in (("concat_piston", {}), ("blend", {"gather_mode": B.GATHER_BLEND, "piston": False})):
        g = B.Letkf([dataclasses.replace(spec, **kw)])
        g.set_schedule(True, True)
        var = []
        for k in range(T):
            g.step(y[k])
            if k >= T // 2:
                var.append(float(torch.var(g.get_mean() - ph[k], unbiased=False)))
        blend[name + "_residual_variance"] = round(float(np.mean(var)), 5)
        g.close()
    out["blend_gather"] = blend
    # covariance localisation (2-pitch taper, pistons) against the local analysis
    cl = {}
    for name, kw in (("cl_taper2", {"localisation": B.LOCALISATION_COVARIANCE, "taper_c": 2.0}),
                     ("cl_untapered", {"localisation": B.LOCALISATION_COVARIANCE, "taper_c": 0.0})):
        g = B.Letkf([dataclasses.replace(spec, **kw)])
        g.set_schedule(True, True)
        if name == "cl_taper2":
            cl["ms_per_step"] = round(time_steps(g, y, K, W), 5)
            g.set_ensemble(torch.zeros(g.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
            g.set_frame(0)
        var = []
        for k in range(T):
            g.step(y[k])
            if k >= T // 2:
                var.append(float(torch.var(g.get_mean() - ph[k], unbiased=False)))
        cl[name + "_residual_variance"] = round(float(np.mean(var)), 5)
        g.close()
    cl["local_analysis_residual_variance"] = blend["concat_piston_residual_variance"]
    out["covariance_localisation"] = cl
    return out


def kf_reference_line(B, wl_mod):
    """Sec. 5 criterion on the seeded 12x12 reference loop: the coherent energy
    of the local ETKF closed loop on the GPU (4x4 domains, halo 1, m = 64,
    pistons, FP32 state) and its loss against the stationary KF's, which
    tests/golden/kf_reference_12x12.json stores (written from the oracle)."""
    import torch
    c = wl_mod.reference_loop()
    N, a = c["n_sub"], c["a"]
    bank = wl_mod.noise_bank(16, 32, c["pitch"], c["r0"], c["L0"], a, np.random.default_rng(7))
    spec = B.InstanceSpec(n_sub=N, m=64, domain_size=4, halo=1, obscuration=0.0,
                          mask=np.ones((N, N), np.uint8), rho=1.05, r_sigma2=c["sigma"] ** 2, ar_coeff=a,
                          noise_bank=bank, seed=99, precision=B.FP32, piston=True, model=B.MODEL_CLOSED_LOOP)
    f = B.Letkf([spec])
    ij = f.geometry(0)["node_ij"]
    ph = torch.from_numpy(np.ascontiguousarray(c["truth"][:, ij[:, 0], ij[:, 1]], dtype=np.float32)).cuda()
    noise = torch.from_numpy(c["noise"].astype(np.float32)).cuda()
    u1 = torch.zeros(ph.shape[1], dtype=torch.float32, device="cuda")
    u2 = u1.clone()
    var = []
    for k in range(1, ph.shape[0]):
        f.step(f.slopes(ph[k - 1] - u2) + noise[k - 1])
        if k > c["burn_in"]:
            var.append(float(torch.var(ph[k] - u1, unbiased=False)))
        u2, u1 = u1, f.get_command()
    f.close()
    e = float(np.exp(-np.mean(var)))
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "kf_reference_12x12.json")))
    return {"system": ref["system"], "frames": ph.shape[0] - 1, "burn_in": c["burn_in"],
            "e_coh_letkf": round(e, 5), "e_coh_kf": round(ref["e_coh_kf"], 5),
            "loss_percent": round((ref["e_coh_kf"] - e) / ref["e_coh_kf"] * 100.0, 3)}


def make_inputs(f, wl_mod, w, frames: int, rng):
    """Slopes of an AR(1) true phase for `frames` frames, resident on the GPU."""
    import torch
    geo = f.geometry(0)
    ij = geo["node_ij"]
    truth = wl_mod.ar1_truth(w.n_sub, frames, w.pitch, w.r0, w.L0, w.a, rng)
    ph = torch.from_numpy(np.ascontiguousarray(truth[:, ij[:, 0], ij[:, 1]], dtype=np.float32)).cuda()
    p = f.sizes["n_slopes"]
    y = torch.empty((frames, p), dtype=torch.float32, device="cuda")
    for k in range(frames):
        f.slopes(ph[k], out=y[k])
    noise = torch.from_numpy(wl_mod.gaussian_noise((frames, p), w.sigma, rng).astype(np.float32)).cuda()
    y += noise
    torch.cuda.synchronize()
    return y, truth, ij


def time_steps(f, y, K, W, plain=False, per_step=False, offset=0):
    """W untimed then K timed steps on slopes y[offset + W + k]."""
    import torch
    step = f.step_plain if plain else f.step
    y = y[offset:] if offset else y
    for k in range(W):
        step(y[k % y.shape[0]])
    torch.cuda.synchronize()
    if per_step:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            ev[k][0].record()
            step(y[(W + k) % y.shape[0]])
            ev[k][1].record()
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in ev])
    if K == 0:
        torch.cuda.synchronize()
        return None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(K):
        step(y[(W + k) % y.shape[0]])
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K


def host_cpu() -> dict:
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


_POOL = {}


def _pool_init(state):
    from threadpoolctl import threadpool_limits
    _POOL.update(state)
    _POOL["limit"] = threadpool_limits(limits=1)


def _pool_domains(idx):
    """Local analyses (L1-L5) of the given domains of the staged frame."""
    from oracle import letkf as ol
    st = _POOL
    prm, doms = st["prm"], st["doms"]
    for k in idx:
        dom = doms[k]
        Y, dl, g = ol.local_inputs(st["G"], dom, st["Yp"], st["d"], st["r"], prm)
        wv, Wm, _, _ = ol.local_weights(Y, dl, g, prm.rho)
        ol.local_update(st["xb"][dom.owned], st["Xp"][dom.owned], wv, Wm, prm.rho)
    return len(idx)


def table2_domain_ms(reps: int = 200) -> float:
    """The oracle's local update of one domain at the paper's Table 2 shape
    (m = 101 members, n = 32 state entries, p = 128 slopes), one thread,
    median over `reps` calls, in ms."""
    from threadpoolctl import threadpool_limits
    from oracle import letkf as ol
    rng = np.random.default_rng(11)
    m, n, p = 101, 32, 128
    Xp = rng.standard_normal((n, m))
    Xp -= Xp.mean(axis=1, keepdims=True)
    Y = rng.standard_normal((p, m))
    Y -= Y.mean(axis=1, keepdims=True)
    d, g, xb = rng.standard_normal(p), np.full(p, 100.0), rng.standard_normal(n)
    ts = []
    with threadpool_limits(limits=1):
        for _ in range(reps):
            t0 = time.perf_counter()
            wv, Wm, _, _ = ol.local_weights(Y, d, g, 1.05)
            ol.local_update(xb, Xp, wv, Wm, 1.05)
            ts.append(time.perf_counter() - t0)
    return float(np.median(ts)) * 1e3


def cpu_baseline(w, bank, seed, truth, sigma_noise, budget_s=10.0, pool_s=8.0):
    """The FP64 oracle on the same workload: full frames on one thread until
    the budget; then the local analyses of one staged frame spread over a
    process pool (one single-threaded process per usable core, at most 16);
    then one domain at the paper's Table 2 shape.  The oracle's slopes are made
    from the same true phase with the oracle's own operator."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import geometry as og
    from oracle import letkf as ol
    from oracle import philox
    G = og.Geometry(og.pupil_mask(w.n_sub, w.obscuration))
    ij0 = G.node_coords()
    y_host = [og.apply_slopes(G, truth[k][ij0[:, 0], ij0[:, 1]]) + sigma_noise[k] for k in range(len(truth))]
    doms = og.domains(G, w.b, w.h)
    prm = ol.Params(a=w.a, rho=w.rho, b=w.b, h=w.h, piston=True)
    r = np.full(G.n_slopes, w.sigma ** 2)
    ij = G.node_coords()
    Xa = np.zeros((G.n_nodes, w.m))
    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while done < 2 or time.perf_counter() - t0 < budget_s:
            V = philox.bank_noise(bank, ij, w.m, seed, 0, done)
            Xa = ol.step(G, doms, Xa, V, y_host[done % len(y_host)], r, prm)
            done += 1
            if done >= len(y_host):
                break
    dt = time.perf_counter() - t0
    # the local analyses of the next frame over a process pool (spawned
    # interpreters: numpy and the oracle only)
    V = philox.bank_noise(bank, ij, w.m, seed, 0, done)
    Xb = ol.forecast(Xa, V, prm.a)
    xb, Xp = ol.ensemble_stats(Xb)
    state = {"G": G, "doms": doms, "prm": prm, "r": r, "xb": xb, "Xp": Xp,
             "Yp": og.apply_slopes(G, Xp), "d": y_host[done % len(y_host)] - og.apply_slopes(G, xb)}
    cpu = host_cpu()
    nproc = max(1, min(16, cpu["usable_cpus"] or 1))
    chunks = [list(range(k, len(doms), nproc)) for k in range(nproc)]
    with mp.get_context("spawn").Pool(nproc, initializer=_pool_init, initargs=(state,)) as pool:
        pool.map(_pool_domains, chunks)          # warm-up (imports, BLAS set-up)
        n_an, t1 = 0, time.perf_counter()
        while n_an == 0 or time.perf_counter() - t1 < pool_s:
            n_an += sum(pool.map(_pool_domains, chunks))
        pool_dt = time.perf_counter() - t1
    per_core = done * len(doms) / dt
    return {"value": done / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} frames of the same 80x80 m=64 workload ({len(doms)} local analyses each, "
                      f"piston step included), NumPy FP64 with LAPACK eigh, one thread, {dt:.1f} s",
            "host": cpu,
            "local_analyses_per_s_1core": round(per_core, 1),
            "all_cores": {"processes": nproc, "local_analyses_per_s": round(n_an / pool_dt, 1),
                          "frames_per_s_analyses_only": round(n_an / pool_dt / len(doms), 2),
                          "sample": f"{n_an} local analyses (L1-L5 of one staged frame, repeated) in "
                                    f"{pool_dt:.1f} s over {nproc} single-threaded processes"},
            "table2_domain": {"shape": "m=101, n=32, p=128", "oracle_ms_1core": round(table2_domain_ms(), 4),
                              "paper_ms": 0.94, "paper_hardware": "1 core of 2x Intel Xeon E5-2680 v2 (Table 2)"}}


def other_workloads(B, wl, K, W, transform):
    """Frame time of the other workloads (graph replay, bank noise, piston
    removal on): the 8x8 FP64 case, the 40x40 frozen-flow case and 64
    independent instances in one launch."""
    import torch
    out = {}
    for idx, label in ((0, "8x8 square m=20 FP64"), (1, "40x40 eps0.14 m=50 frozen flow"),
                       (3, "64 instances N~U{16..48}, m in {32,48,64}")):
        ws = wl.workloads(idx)
        rng = np.random.default_rng(ws[0].seed)
        specs, ys = [], []
        frames = K + W
        for i, w in enumerate(ws):
            bank = wl.bank_for(w, rng, n_screens=8)
            specs.append(B.InstanceSpec(n_sub=w.n_sub, m=w.m, domain_size=w.b, halo=w.h,
                                        obscuration=0.0 if w.obscuration is None else w.obscuration,
                                        mask=np.ones((w.n_sub, w.n_sub), bool) if w.obscuration is None else None,
                                        rho=w.rho, r_sigma2=w.sigma ** 2, ar_coeff=w.a, noise_bank=bank,
                                        seed=0x5EED0000 + w.seed + i,
                                        precision=B.FP64 if w.precision == "fp64" else B.FP32, piston=True,
                                        transform=transform))
        f = B.Letkf(specs)
        dt = torch.float64 if f.fp64 else torch.float32
        y = torch.empty((frames, f.sizes["n_slopes"]), dtype=dt, device="cuda")
        phase = torch.empty(f.sizes["n_nodes"], dtype=dt, device="cuda")
        truths = [wl.truth_for(w, rng, frames=frames) for w in ws]
        node_ij = [f.geometry(i)["node_ij"] for i in range(len(ws))]
        for k in range(frames):
            ph = np.concatenate([truths[i][k][node_ij[i][:, 0], node_ij[i][:, 1]] for i in range(len(ws))])
            phase.copy_(torch.from_numpy(ph.astype(np.float64 if f.fp64 else np.float32)))
            f.slopes(phase, out=y[k])
            y[k] += torch.randn(f.sizes["n_slopes"], dtype=dt, device="cuda") * float(ws[0].sigma)
        ms = time_steps(f, y, K, W)
        row = {"instances": len(ws), "domains": int(f.sizes["n_domains"]),
               "ms_per_step": round(ms, 4), "frames_per_s": round(1000.0 / ms, 1),
               "local_analyses_per_s": round(f.sizes["n_domains"] * 1000.0 / ms, 1)}
        if not f.fp64:
            # the analysis kernel's own duration, and the roofline fraction with
            # each instance's own m, p_l and n_l
            f.set_schedule(False, 1)
            f.set_timing(True)
            time_steps(f, y, K, 0)
            kt = float(np.mean(f.analysis_times()))
            f.set_timing(False)
            t_lb, _ = handle_bound(f)
            row.update({"kernel_ms": round(kt, 4), "t_lb_us": round(t_lb * 1e6, 3),
                        "frac_kernel": round(t_lb / (kt * 1e-3), 4), "frac_frame": round(t_lb / (ms * 1e-3), 4)})
        out[label] = row
        f.close()
    return out


def gradient_timing(B, w, bank, seed, y, truth, ij, T):
    """The tuning run's gradient: T frames of the 80x80 workload with a
    Gaspari-Cohn taper (c = 2 pitches), loss = mean residual variance, gradient
    in (rho, r_scale, taper_c) through the hand-written adjoint, checkpoints
    every 20 frames."""
    import torch
    from paper_1408_7069_amd import tuning
    spec = B.InstanceSpec(n_sub=w.n_sub, m=w.m, domain_size=w.b, halo=w.h, obscuration=w.obscuration,
                          rho=w.rho, r_sigma2=w.sigma ** 2, ar_coeff=w.a, noise_bank=bank, seed=seed,
                          taper_c=2.0, precision=B.FP32, piston=True)
    f = B.Letkf([spec])
    T = min(T, y.shape[0])
    ts = [torch.from_numpy(np.ascontiguousarray(truth[k][ij[:, 0], ij[:, 1]], dtype=np.float32)).cuda()
          for k in range(T)]
    ys = [y[k] for k in range(T)]
    theta = torch.tensor([w.rho, 1.0, 2.0], dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = tuning.residual_variance_loss(f, theta, ys, ts, checkpoint_every=20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.sum().backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f.close()
    return {"frames": T, "checkpoint_every": 20, "forward_s": round(t1 - t0, 4),
            "backward_s": round(t2 - t1, 4), "loss": loss.item(),
            "d_loss_d_rho_rscale_taper": [float(v) for v in theta.grad],
            "note": "80x80 m=64 with taper c=2; FP32 state, FP64 eigensolve and its adjoint"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--copies", default="1,4,16,64",
                    help="comma list: instances of the workload in one launch (batched throughput lines)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--transform", default="nsp_mixed", choices=list(TRANSFORMS),
                    help="transform of the local analyses in the headline frame")
    ap.add_argument("--quick", action="store_true",
                    help="headline frame, batched copies and transforms only (no loops, no CPU leg)")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3: timed steps only")
    ap.add_argument("--grad-frames", type=int, default=200, help="frames of the gradient timing (0 = skip)")
    ap.add_argument("--other-workloads", type=int, default=1, help="also time the 8x8, 40x40 and 64-instance workloads")
    ap.add_argument("--paper-shape", type=int, default=1,
                    help="also time the paper's timing shape (m = 101, halo 2) on the 80x80 pupil")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the frame is not sharded "
              "across GPUs in this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1408_7069_amd import binding as B
    from paper_1408_7069_amd import workload as wl

    torch.cuda.init()
    w = wl.workloads(2)[0]
    rng = np.random.default_rng(w.seed)
    bank = wl.bank_for(w, rng, n_screens=16)
    seed = 0x5EED0000 + w.seed
    spec = B.InstanceSpec(n_sub=w.n_sub, m=w.m, domain_size=w.b, halo=w.h, obscuration=w.obscuration,
                          rho=w.rho, r_sigma2=w.sigma ** 2, ar_coeff=w.a, noise_bank=bank, seed=seed,
                          precision=B.FP32, piston=True, transform=getattr(B, TRANSFORMS[args.transform]))
    f = B.Letkf([spec])
    K, W = args.steps, args.warmup
    frames = min(K + W, 600)
    y, truth, ij = make_inputs(f, wl, w, frames, rng)
    print(f"# inputs ready: {frames} frames of slopes on the GPU", file=sys.stderr, flush=True)

    if args.profile:
        # direct launches (the same kernel the graph replays), then a plain
        # copy of known size that calibrates the HBM byte counters
        f.set_schedule(False, True)
        time_steps(f, y, K, W)
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "steps": K, "copy_bytes": COPY_BYTES}))
        return

    sched = f.autotune(y[0], frames=50)
    f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    f.set_frame(0)
    ms = time_steps(f, y, K, W)
    fps = 1000.0 / ms
    # the filter is tracking: residual variance of the last analysis mean
    last = (W + K - 1) % y.shape[0]
    t_last = truth[last][ij[:, 0], ij[:, 1]].astype(np.float64)
    e = f.get_mean().cpu().numpy().astype(np.float64) - t_last
    filt = {"frame": last, "residual_variance": float(np.mean((e - e.mean()) ** 2)),
            "phase_variance": float(np.mean((t_last - t_last.mean()) ** 2))}
    n_dom = f.sizes["n_domains"]
    # per-step distribution (graph replay), then the analysis kernel's own
    # launch duration from HIP events around it (direct launches, same kernel)
    f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    f.set_frame(0)
    per = time_steps(f, y, K, W, per_step=True)
    f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    f.set_frame(0)
    f.set_schedule(False, sched[1])
    time_steps(f, y, 0, W)
    f.set_timing(True)
    time_steps(f, y, K, 0, offset=W)
    kt = f.analysis_times()
    f.set_timing(False)
    f.set_schedule(*sched)
    kernel_ms = float(np.mean(kt))
    # plain form: one launch per domain, no graph, on the same frames
    f.set_ensemble(torch.zeros(f.sizes["ensemble_elems"], dtype=torch.float32, device="cuda"))
    f.set_frame(0)
    time_steps(f, y, 0, W)
    plain_ms = time_steps(f, y, args.plain_steps, 0, plain=True, offset=W)

    # roofline of the analysis kernel: the counted work's lower-bound time at
    # the MI355X peaks over the kernel's own duration (HIP events around its
    # direct launches; the committed rocprofv3 trace's average beside it)
    t_lb, fl = handle_bound(f)
    g = f.geometry(0)
    fl_all = algorithmic_flops(w.m, np.diff(g["obs_off"]), np.diff(g["own_off"]))
    # achieved in FP64-equivalent TFLOP/s: the FP32 matrix-core work counted
    # at half weight (its peak is twice the FP64 one), so achieved / 78.6 is
    # exactly sum(T_lb) / t_kernel
    fp64_equiv = fl["evd_fp64"] + 0.5 * (fl["gram_fp32"] + fl["update_fp32"])
    achieved = fp64_equiv / (kernel_ms * 1e-3) / 1e12
    tr_ms = trace_kernel_ms()
    steps = (f.status()[1] >> 8) & 255
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic(),
            "kernel": f"k_analysis<float,true,{transform_name(B, spec.transform)}>",
            "kernel_ms_events": round(kernel_ms, 4),
            "kernel_ms_trace": None if tr_ms is None else round(tr_ms, 4),
            "frac_trace": None if tr_ms is None else round(t_lb / (tr_ms * 1e-3), 4),
            "frac_frame": round(t_lb / (ms * 1e-3), 4),
            "t_lb_us": round(t_lb * 1e6, 3),
            "counted_flops": fl, "not_counted_flops": fl_all["not_counted"],
            "achieved_note": "FP64-equivalent: EVD 9m^3/domain at the FP64 peak plus Gram and "
                             "update at half weight (FP32 matrix-core peak 157.3 = 2 x 78.6)",
            "transform_steps_mean": round(float(steps.mean()), 3)}

    # batched throughput: copies of the workload in one launch (per-domain
    # cost does not depend on the telescope, so copies are the batch axis)
    batched = []
    for nc in ([int(c) for c in args.copies.split(",") if c] if args.copies else []):
        batched.append(batched_line(B, spec, y, min(K, 100), W, nc))

    others = (other_workloads(B, wl, max(20, min(K, 100)), W, spec.transform)
              if args.other_workloads else None)

    transforms = transform_variants(B, spec, y, K, W, args.transform)
    paper_shape = paper_shape_lines(B, w, bank, seed, y, min(K, 100), W) if args.paper_shape else None
    loop = kfref = models = None
    if not args.quick:
        loop = closed_loop_line(B, spec, wl, w, y, truth, ij, K, W)
        kfref = kf_reference_line(B, wl)
        models = model_variants(B, spec, wl, w, y, truth, ij, K, W)

    grad = None
    if args.grad_frames > 0 and not args.quick:
        grad = gradient_timing(B, w, bank, seed, y, truth, ij, args.grad_frames)

    out = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "80x80 SH, 28% obscuration, m=64, 4x4-subaperture domains, halo 1: "
                               f"{n_dom} local analyses per frame in one launch ({schedule_label(sched)}), "
                               f"transform {transform_name(B, spec.transform)}",
                   "n_slopes": int(f.sizes["n_slopes"]), "n_nodes": int(f.sizes["n_nodes"]),
                   "domains": int(n_dom), "schedule": {"graph": bool(sched[0]), "order": int(sched[1])}},
        "local_analyses_per_s": round(fps * n_dom, 1),
        "plain": {"ms_per_step": round(plain_ms, 4), "frames_per_s": round(1000.0 / plain_ms, 2),
                  "launches_per_step": int(n_dom)},
        "step_ms_p50": round(float(np.percentile(per, 50)), 4),
        "step_ms_p99": round(float(np.percentile(per, 99)), 4),
        "batched_copies": batched,
        "transforms": transforms,
        "paper_shape": paper_shape,
        "closed_loop": loop,
        "kf_reference": kfref,
        "model_variants": models,
        "filter_check": filt,
        "other_workloads": others,
        "gradient": grad,
        "roofline": roof,
    }
    if not args.no_cpu and not args.quick:
        nrng = np.random.default_rng(w.seed + 1)
        T = min(frames, 400)   # more frames than the time budget reaches
        out["cpu_baseline"] = cpu_baseline(w, bank, seed, truth[:T],
                                           wl.gaussian_noise((T, f.sizes["n_slopes"]), w.sigma, nrng))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
