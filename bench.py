#!/usr/bin/env python3
"""Throughput of the batched RTO posterior sampler on one MI355X.

One step = one pass of the whole hot path over one batch: 64 RTO samples of the
195,112-node mapped-ball problem (1000 leapfrog steps, 1024 sensors), each the
100-iteration CGLS solve of the perturbed least-squares problem, run as one
multi-RHS block with float32 sweeps and float64 CGLS vectors, dots and scalars,
followed by the posterior mean and standard deviation.  Inputs (mesh operators,
data, perturbations) are resident on the GPU before the timed region.

Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def step_bytes(info, RB, tsize, kind):
    """Algorithmic HBM bytes of one step launch (each array element read or written once).

    Both steps carry the three-level state: S^n read (its rows also serve as the neighbours),
    S^{n-1} read and S^{n+1} written.
    forward : CSR (col + value), rowptr, boundary offsets, dt/m, stored boundary values, the
              state, sensor rows and the float64 sample output.
    transpose: same matrix data and state plus the injection CSR, and the float64 data values of
              two sample times injected at the sensor nodes.
    """
    N, nnz, nobs = info["n_nodes"], info["nnz_k"], info["n_obs"]
    b = nnz * (4 + tsize) + (N + 1) * 4 + N * 4 + N * tsize + info["b_stored"] * tsize
    b += 3 * N * RB * tsize
    if kind == "fwd":
        b += nobs * 4 * (4 + tsize) + nobs * RB * 8
    else:
        b += (N + 1) * 4 + 4 * nobs * (4 + tsize) + 2 * 4 * nobs * RB * 8
    return int(b)


def kernel_source_sha():
    """Hash of what decides the step kernels' memory traffic: their code, their work mappings and
    the host setup that lays out and orders the rows (comments and layout whitespace left out)."""
    h = hashlib.sha256()
    for name in ("pat_kernels.hip", "pat_tiles.h", "pat_setup.cpp"):
        with open(os.path.join(ROOT, "paper_2607_21373_amd", "csrc", name)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def stored_traffic(kernel, workload):
    """HBM traffic of the step kernel from the committed rocprofv3 counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d[kernel][workload]
        if e.get("kernels_sha") != kernel_source_sha():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(w, eta, xi, yobs, sigma, n_iter, R, n_steps_sample=350, iters_sample=3, reorth_iters=6,
                 reorth_steps=10):
    """Oracle (plain CPU FP64) on a bounded sample of the same workload, extrapolated to the full batch.

    The sweeps scale with sweep-steps; the reorthogonalisation of iteration j projects against j basis
    vectors, so its cost grows with the iteration count.  It is measured on its own: two short runs
    (reorth_iters iterations over reorth_steps steps, with and without reorthogonalisation) give the
    cost of one basis-vector pass, and the full batch adds that cost times 1 + 2 + ... + n_iter."""
    import oracle
    t0 = time.time()
    P = oracle.Problem.from_workload(w, n_steps=n_steps_sample)
    setup = time.time() - t0
    t0 = time.time()
    P.rto(yobs[:n_steps_sample], sigma, w.prior_a, iters_sample, eta[:R, :n_steps_sample], xi[:R])
    el = time.time() - t0
    # the reorthogonalisation's cost per basis vector, from a short run with and without it
    Pr = oracle.Problem.from_workload(w, n_steps=reorth_steps)
    t0 = time.time()
    Pr.rto(yobs[:reorth_steps], sigma, w.prior_a, reorth_iters, eta[:R, :reorth_steps], xi[:R], reorth=True)
    t_on = time.time() - t0
    t0 = time.time()
    Pr.rto(yobs[:reorth_steps], sigma, w.prior_a, reorth_iters, eta[:R, :reorth_steps], xi[:R], reorth=False)
    t_off = time.time() - t0
    per_vec = max(t_on - t_off, 0.0) / (reorth_iters * (reorth_iters + 1) / 2)
    sweeps_sample = 2 * iters_sample
    sweeps_full = 2 * n_iter
    t_sweeps = (el - per_vec * iters_sample * (iters_sample + 1) / 2) * (sweeps_full / sweeps_sample) * \
        (w.n_steps / n_steps_sample)
    t_reorth = per_vec * n_iter * (n_iter + 1) / 2
    t_batch = t_sweeps + t_reorth
    return {
        "value": round(R / t_batch * 60.0, 6), "unit": "samples/min", "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"oracle RTO on the same mesh with {R} RHS: {iters_sample} CGLS iterations x {n_steps_sample} "
                   f"steps ({el:.1f} s, setup {setup:.1f} s excluded) scaled by sweep-steps to {n_iter} iterations x "
                   f"{w.n_steps} steps ({t_sweeps:.0f} s), plus the reorthogonalisation measured from "
                   f"{reorth_iters}-iteration runs over {reorth_steps} steps with and without it "
                   f"({t_on:.1f} / {t_off:.1f} s: {per_vec:.3f} s per basis-vector pass) grown to {n_iter} "
                   f"iterations ({t_reorth:.0f} s)"),
        "extrapolated_batch_s": round(t_batch, 1),
    }


def _synth(pat, W, w, G, dev):
    """Noisy data from the library's float64 forward map (the paper's relative-L2 noise rule)."""
    import torch
    p0 = torch.as_tensor(w.p0_true, dtype=torch.float64, device=dev)[None].contiguous()
    Y = pat.pat_forward(G, p0)[0]
    eta0 = torch.as_tensor(W.noise_draw(w.n_steps, w.n_obs, w.noise_seed), device=dev)
    sigma = float(w.d_noise * torch.linalg.norm(Y) / torch.linalg.norm(eta0))
    return (Y + sigma * eta0).contiguous(), sigma


def uneven_leg(pat, W, dev, n_iter, modes=False, names=("cube40", "ball60", "slab120")):
    """Meshes of different sizes sampled together (rto_sample_batch, autotuned launch mode),
    16 samples each with device-drawn perturbations, against the same solves run one
    after another with the same RHS block."""
    import torch
    ws = [W.make_workload(n) for n in names]
    t0 = time.time()
    probs = [pat.Problem.from_workload(w) for w in ws]
    log(f"uneven batch: {', '.join(f'{w.name} N={w.n_nodes}' for w in ws)} set up in {time.time() - t0:.1f} s")
    data = [_synth(pat, W, w, G, dev) for w, G in zip(ws, probs)]
    B = pat.Batch(probs)
    S = 16
    rb, us = B.autotune(S, "f32")
    log(f"uneven batch: autotuned RHS block {rb} (priced {us:.1f} us per merged forward+transpose step)")

    def batched():
        return pat.rto_sample_batch(B, [d[0] for d in data], None, None, [d[1] for d in data],
                                    [w.prior_a for w in ws], n_iter, sweep_prec="f32", n_samples=S, seed=17)

    def serial():
        return [pat.rto_sample(G, d[0], None, None, d[1], w.prior_a, n_iter, sweep_prec="f32", rhs_block=rb,
                               n_samples=S, seed=17) for w, G, d in zip(ws, probs, data)]

    batched()
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = batched()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    serial()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ref = serial()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    same = all(torch.equal(a["samples"], b["samples"]) for a, b in zip(outs, ref))
    mode_times = {}
    if modes:
        # each launch mode of pat_batch_merge forced for both directions (1 merged per step,
        # 0 one launch per mesh per step, 2 whole sweep per mesh), then back to the tuned choice
        for m in (1, 0, 2):
            B.merge(m, m)
            batched()
            torch.cuda.synchronize()
            t = time.perf_counter()
            batched()
            torch.cuda.synchronize()
            mode_times[{1: "merged_per_step", 0: "per_mesh_per_step", 2: "whole_sweep_per_mesh"}[m]] = \
                round(time.perf_counter() - t, 3)
        B.merge(-1, -1)
        log(f"uneven batch launch modes: {mode_times}")
    res = {"meshes": {w.name: w.n_nodes for w in ws}, "samples": S * len(ws), "iters": n_iter, "rhs_block": rb,
           "seconds": round(tb, 3), "value": round(S * len(ws) / tb * 60.0, 3), "unit": "samples/min",
           "serial_seconds": round(ts, 3), "speedup_vs_serial": round(ts / tb, 3), "equal_to_serial": same}
    if mode_times:
        res["mode_seconds"] = mode_times
    log(f"uneven batch: {tb:.2f} s for {S * len(ws)} samples ({res['value']:.1f} samples/min); one mesh after "
        f"another {ts:.2f} s; results identical: {same}")
    return res


def big_leg(pat, W, dev, n_iter):
    """One sample on the 10^6-node ball: float32 sweeps and the plain float64 path."""
    import torch
    w = W.make_workload("ball100")
    t0 = time.time()
    G = pat.Problem.from_workload(w)
    info = G.info()
    log(f"ball100: N={w.n_nodes} nnz={info['nnz_k']} set up in {time.time() - t0:.1f} s")
    yobs, sigma = _synth(pat, W, w, G, dev)
    res = {"n_nodes": w.n_nodes, "n_steps": w.n_steps, "iters": n_iter}
    for prec in ("f32", "f64"):
        G.profile_enable(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        pat.rto_sample(G, yobs, None, None, sigma, w.prior_a, n_iter, sweep_prec=prec, rhs_block=1, n_samples=1,
                       seed=1, stats=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        prof = G.profile()
        G.profile_enable(False)
        tsz = 4 if prec == "f32" else 8
        fwd_s = prof["fwd_ms"] / max(prof["fwd_sweeps"], 1) / w.n_steps / 1e3
        gbs = step_bytes(info, 1, tsz, "fwd") / fwd_s / 1e9
        res[prec] = {"seconds_per_sample": round(el, 3), "samples_per_min": round(60.0 / el, 3),
                     "fwd_step_us": round(fwd_s * 1e6, 3), "fwd_step_GBs": round(gbs, 1)}
        log(f"ball100 {prec}: {el:.2f} s per sample; forward step {fwd_s * 1e6:.1f} us ({gbs:.0f} GB/s)")
    # 64 float32 RHS per sweep: the state of a step (1 GB) no longer fits the Infinity Cache
    p0 = torch.randn(64, w.n_nodes, dtype=torch.float32, device=dev)
    y = pat.pat_forward(G, p0)
    a = pat.pat_adjoint(G, y)
    r64 = {}
    for name, fn, kind in (("fwd", lambda: pat.pat_forward(G, p0, y), "fwd"),
                           ("adj", lambda: pat.pat_adjoint(G, y, a), "adj")):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 2 / w.n_steps * 1e3
        r64[f"{name}_step_us"] = round(us, 2)
        r64[f"{name}_step_GBs"] = round(step_bytes(info, 64, 4, kind) / us / 1e3, 1)
    res["rhs64_sweeps"] = r64
    log(f"ball100, 64 float32 RHS per sweep: {r64} (per step, including the layout conversion of the entry points)")
    return res


def roofline_record(fwd_s, adj_s, fb, ab, survey_bytes, sweep_share, wname, RB):
    """Roofline of the two step kernels, which share the sweep time almost equally: the one with the
    longer average launch leads the record, the other follows with its own fraction of the HBM peak."""
    # float32 blocks of 64, 128 or 256 RHS run the halo-tile step kernels, narrower ones the vector-lane ones
    fk, ak = (f"k_fwd_h<double,{RB}>", f"k_adj_h<double,{RB}>") if RB >= 64 else \
        (f"k_fwd_v<float,double,{RB}>", f"k_adj_v<float,double,{RB}>")
    kern = {"fwd": (f"{fk} (forward leapfrog step)", fwd_s, fb, f"k_fwd_f32_rb{RB}"),
            "adj": (f"{ak} (transpose leapfrog step)", adj_s, ab, f"k_adj_f32_rb{RB}")}

    def rec(k):
        name, sec, b, key = kern[k]
        gbs = b / sec / 1e9
        r = {"kernel": name, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": stored_traffic(key, wname),
             "bytes_per_launch": b, "avg_launch_us": round(sec * 1e6, 3)}
        if survey_bytes:
            r["frac_survey_bytes"] = round(survey_bytes / sec / 1e9 / HBM_PEAK_GBS, 4)
        return r

    lead, other = ("adj", "fwd") if adj_s >= fwd_s else ("fwd", "adj")
    out = rec(lead)
    out["co_dominant"] = rec(other)
    out["sweep_time_share"] = round(sweep_share, 4)
    if survey_bytes:
        out["survey_bytes_per_sweep_step"] = survey_bytes
    return out


def wide_probe(pat, G, info, w, yobs, sigma, iters=4):
    """The step kernels with 256 samples as one 256-RHS block on the same mesh: the float32 state of a
    step (4 x N x 256 x 4 B = 800 MB) no longer fits the 256 MB Infinity Cache.  A short solve
    (a few iterations) gives the average launch of both steps."""
    import torch
    RB = 256
    args = (G, yobs, None, None, sigma, w.prior_a)
    pat.rto_sample(*args, 1, sweep_prec="f32", rhs_block=RB, n_samples=RB, seed=11, stats=False)
    G.profile_enable(True)
    torch.cuda.synchronize()
    pat.rto_sample(*args, iters, sweep_prec="f32", rhs_block=RB, n_samples=RB, seed=11, stats=False)
    torch.cuda.synchronize()
    prof = G.profile()
    G.profile_enable(False)
    fwd_s = prof["fwd_ms"] / max(prof["fwd_sweeps"], 1) / w.n_steps / 1e3
    adj_s = prof["adj_ms"] / max(prof["adj_sweeps"], 1) / w.n_steps / 1e3
    fb, ab = step_bytes(info, RB, 4, "fwd"), step_bytes(info, RB, 4, "adj")
    res = {"rhs_block": RB, "state_MB": round(3 * w.n_nodes * RB * 4 / 1e6, 1)}
    for k, sec, b in (("fwd", fwd_s, fb), ("adj", adj_s, ab)):
        gbs = b / sec / 1e9
        res[k] = {"avg_launch_us": round(sec * 1e6, 3), "bytes_per_launch": b, "achieved": round(gbs, 1),
                  "frac": round(gbs / HBM_PEAK_GBS, 4),
                  "traffic": stored_traffic(f"k_{k}_f32_rb{RB}", w.name)}
    log(f"256-RHS block steps: forward {fwd_s * 1e6:.1f} us ({res['fwd']['achieved']:.0f} GB/s), transpose "
        f"{adj_s * 1e6:.1f} us ({res['adj']['achieved']:.0f} GB/s)")
    return res


def wide_leg(pat, dev, G, info, w, yobs, sigma, n_iter):
    """256 samples as one 256-RHS block on the same mesh: the float32 state of a step
    (4 x N x 256 x 4 B = 800 MB) no longer fits the 256 MB Infinity Cache."""
    import torch
    S = RB = 256
    args = (G, yobs, None, None, sigma, w.prior_a)
    pat.rto_sample(*args, 2, sweep_prec="f32", rhs_block=RB, n_samples=S, seed=11)  # graphs and workspaces
    G.profile_enable(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    pat.rto_sample(*args, n_iter, sweep_prec="f32", rhs_block=RB, n_samples=S, seed=11)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    prof = G.profile()
    G.profile_enable(False)
    # as in the main leg: sweep time over N_T step launches (the extra init/sampling launch is tiny)
    fwd_s = prof["fwd_ms"] / max(prof["fwd_sweeps"], 1) / w.n_steps / 1e3
    adj_s = prof["adj_ms"] / max(prof["adj_sweeps"], 1) / w.n_steps / 1e3
    fb, ab = step_bytes(info, RB, 4, "fwd"), step_bytes(info, RB, 4, "adj")
    res = {"samples": S, "rhs_block": RB, "iters": n_iter, "seconds": round(el, 3),
           "value": round(S * 60.0 / el, 3), "unit": "samples/min",
           "fwd_step_us": round(fwd_s * 1e6, 3), "fwd_step_GBs": round(fb / fwd_s / 1e9, 1),
           "adj_step_us": round(adj_s * 1e6, 3), "adj_step_GBs": round(ab / adj_s / 1e9, 1),
           "bytes_per_fwd_launch": fb, "traffic_per_fwd_launch": stored_traffic("k_fwd_f32_rb256", w.name)}
    log(f"wide block: {S} samples as one {RB}-RHS block in {el:.2f} s ({res['value']:.1f} samples/min); forward "
        f"step {fwd_s * 1e6:.1f} us ({res['fwd_step_GBs']:.0f} GB/s), transpose {adj_s * 1e6:.1f} us")
    return res


def spectral_leg(pat, dev, G, w, yobs, sigma, n_iter):
    """RTO with the Whittle-Matern spectral prior (latent-space solve, Sec. 6.4 construction) on the same
    mesh: 128^3 grid on [-1.25, 1.25)^3, ell = 0.075, prior sigma 3, 64 samples as one 64-RHS block."""
    import torch
    n, lo, side, ell, psig = 128, -1.25, 2.5, 0.075, 3.0
    pat.spectral_prior_set(G, n, lo, side, ell, psig)
    try:
        S = RB = 64
        args = (G, yobs, None, None, sigma, 0.0)
        pat.rto_sample(*args, 2, sweep_prec="f32", rhs_block=RB, n_samples=S, seed=21, prior="spectral")
        # P and P^T alone on 64 RHS (including the binding's layout conversion in and out)
        x = torch.randn(RB, n ** 3, dtype=torch.float64, device=dev)
        v = torch.randn(RB, w.n_nodes, dtype=torch.float64, device=dev)
        pat.spectral_apply(G, x)
        pat.spectral_apply(G, v, transpose=True)
        times = {}
        for name, fn in (("P", lambda: pat.spectral_apply(G, x)), ("PT", lambda: pat.spectral_apply(G, v, True))):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                fn()
            e1.record()
            torch.cuda.synchronize()
            times[name] = e0.elapsed_time(e1) / 3
        del x, v
        # five passes per application on the half spectrum (n/2 + 1 x frequencies): real in / half complex
        # out, three half-complex passes, half complex in / real out
        fft_bytes = int((8 + 16 * (n // 2 + 1) / n + 3 * 32 * (n // 2 + 1) / n + 16 * (n // 2 + 1) / n + 8) * n ** 3 * RB)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = pat.rto_sample(*args, n_iter, sweep_prec="f32", rhs_block=RB, n_samples=S, seed=21, prior="spectral")
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ok = bool(torch.isfinite(out["samples"]).all())
    finally:
        pat.spectral_prior_set(G, None, 0, 0, 0, 0)
    res = {"grid": n, "samples": S, "rhs_block": RB, "iters": n_iter, "seconds": round(el, 3),
           "value": round(S * 60.0 / el, 3), "unit": "samples/min", "finite": ok,
           "P_ms": round(times["P"], 3), "PT_ms": round(times["PT"], 3), "fft_bytes_per_apply": fft_bytes,
           "P_fft_GBs_upper": round(fft_bytes / (times["P"] * 1e-3) / 1e9, 1)}
    log(f"spectral prior: {S} samples in {el:.2f} s ({res['value']:.1f} samples/min); P {times['P']:.2f} ms, "
        f"P^T {times['PT']:.2f} ms per application on {RB} RHS ({fft_bytes / 1e9:.1f} GB of FFT passes)")
    return res


def lsqr_leg(pat, G, w, yobs, eta, xi, sigma, n_iter, R):
    """The main workload solved with LSQR instead of CGLS (same iterates in exact arithmetic)."""
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    pat.rto_sample(G, yobs, eta, xi, sigma, w.prior_a, n_iter, sweep_prec="f32", rhs_block=64, solver="lsqr")
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    res = {"samples": R, "iters": n_iter, "seconds": round(el, 3), "value": round(R * 60.0 / el, 3),
           "unit": "samples/min"}
    log(f"LSQR: {R} samples in {el:.2f} s ({res['value']:.1f} samples/min)")
    return res


def map_leg(G, w, dev, yobs, sigma, iters=50):
    """MAP by gradient descent through the autograd operator (forward = G, backward = G^T) on the same mesh:
    each iteration is one float64 forward and one transpose sweep plus the prior terms."""
    import torch
    from paper_2607_21373_amd import autograd as ag
    y = yobs.contiguous()
    lam = ag.hessian_lambda_max(G, sigma, w.prior_a, iters=5)
    ag.map_gradient_descent(G, y, sigma, w.prior_a, n_iter=2, step=1.0 / (1.02 * lam))
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, hist, _ = ag.map_gradient_descent(G, y, sigma, w.prior_a, n_iter=iters, step=1.0 / (1.02 * lam), history=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    res = {"iters": iters, "seconds": round(el, 3), "ms_per_iter": round(el / iters * 1e3, 3),
           "objective_first_last": [hist[0], hist[-1]]}
    log(f"MAP gradient descent through autograd: {iters} iterations in {el:.2f} s ({res['ms_per_iter']:.2f} ms each)")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ball58_batched")
    ap.add_argument("--iters", type=int, default=None, help="CGLS iterations (default: the workload's 100)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain float64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before timing, copy a float32 buffer of this many MB three times (counter calibration)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="time a plain elementwise update over four state-sized float32 arrays (what streaming "
                         "reaches for the step's working set) and over arrays 8x larger (past the 256 MB cache)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the three-mesh uneven batch")
    ap.add_argument("--no-wide-probe", action="store_true",
                    help="skip the short 256-RHS solve that times the step kernels beyond the Infinity Cache")
    ap.add_argument("--wide-iters", type=int, default=4, help="solver iterations of that 256-RHS solve")
    ap.add_argument("--big", action="store_true", help="also time one sample on the 10^6-node ball")
    ap.add_argument("--spectral", action="store_true",
                    help="also time 64 samples with the Whittle-Matern spectral prior (128^3 grid, latent solve)")
    ap.add_argument("--lsqr", action="store_true", help="also time the main batch solved with LSQR")
    ap.add_argument("--map", action="store_true", help="also time MAP gradient descent through the autograd operator")
    ap.add_argument("--wide", action="store_true",
                    help="also time 256 samples as one 256-RHS block (working set beyond the Infinity Cache)")
    ap.add_argument("--uneven-modes", action="store_true", help="also time each launch mode of the uneven batch")
    ap.add_argument("--uneven-set", default="cube40,ball60,slab120",
                    help="workloads of the uneven batch (equal step counts), comma-separated")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (samples are independent, so "
              "N GPUs would each run their own batches)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2607_21373_amd import pat

    dev = torch.device("cuda", 0)
    w = W.make_workload(args.workload)
    n_iter = args.iters or w.n_iter
    R = w.n_samples
    log(f"workload {w.name}: N={w.n_nodes} E={w.tets.shape[0]} N_T={w.n_steps} N_obs={w.n_obs} R={R} iters={n_iter}")
    t0 = time.time()
    G = pat.Problem.from_workload(w)
    info = G.info()
    log(f"libpat problem created in {time.time() - t0:.1f} s: nnz={info['nnz_k']} "
        f"boundary nodes={info['n_boundary_nodes']} lambda_max={info['lambda_max']:.4g}")

    # synthetic data from the library's own float64 forward map (same recipe as the tests)
    p0 = torch.as_tensor(w.p0_true, dtype=torch.float64, device=dev)[None].contiguous()
    Y = pat.pat_forward(G, p0)[0]
    eta0 = torch.as_tensor(W.noise_draw(w.n_steps, w.n_obs, w.noise_seed), device=dev)
    sigma = float(w.d_noise * torch.linalg.norm(Y) / torch.linalg.norm(eta0))
    yobs = (Y + sigma * eta0).contiguous()
    eta_h, xi_h = W.rto_draws(R, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
    eta = torch.as_tensor(eta_h, device=dev)
    xi = torch.as_tensor(xi_h, device=dev)
    torch.cuda.synchronize()
    log(f"data ready: sigma={sigma:.4e}")

    copy_probe = None
    if args.copy_probe_mb:
        # device-to-device copies of a known size: counter calibration and the practical
        # read+write bandwidth of the memory system
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        e0.record()
        for _ in range(3):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 3 / 1e3
        copy_probe = {"mib": args.copy_probe_mb, "GBs_read_plus_write": round(2 * n * 4 / sec / 1e9, 1)}
        del src, dst
        log(f"copy probe: {args.copy_probe_mb} MiB float32 copies at {copy_probe['GBs_read_plus_write']} GB/s "
            f"(read + write)")

    stream_probe = None
    if args.stream_probe:
        # V' = V - c P, P' = P + c V' with torch's elementwise kernels on arrays of the
        # step's state size (N x 64 float32): 6 array passes per update, no gathers
        stream_probe = {}
        for label, scale, reps in (("state_size", 1, 200), ("state_size_x8", 8, 25)):
            n = scale * w.n_nodes * R
            P, V = torch.ones(n, dtype=torch.float32, device=dev), torch.ones(n, dtype=torch.float32, device=dev)
            P2, V2 = torch.empty_like(P), torch.empty_like(P)

            def upd():
                torch.add(V, P, alpha=-1e-3, out=V2)
                torch.add(P, V2, alpha=1e-3, out=P2)

            upd()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                upd()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / reps / 1e3
            stream_probe[label] = {"array_MB": round(n * 4 / 1e6, 1), "GBs": round(6 * n * 4 / sec / 1e9, 1)}
            del P, V, P2, V2
        log(f"stream probe: {stream_probe}")

    def run():
        # final=True: the float64 recomputation of ||b - G_ext p|| of every sample (one float64
        # forward sweep per block) is part of the timed step
        return pat.rto_sample(G, yobs, eta, xi, sigma, w.prior_a, n_iter, sweep_prec="f32", rhs_block=64,
                              final=True)

    for k in range(args.warmup):
        t = time.time()
        run()
        log(f"warmup {k + 1}/{args.warmup}: {time.time() - t:.2f} s")
    G.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = run()
        log(f"step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = G.profile()
    G.profile_enable(False)
    ms_per_step = el / args.steps * 1e3
    value = R * args.steps / el * 60.0
    mean_norm = float(torch.linalg.norm(out["mean"]))
    fres = out["final_resid"]
    # ||b - G_ext p|| of each sample recomputed in float64; sqrt(N_T N_obs + N) is the size of b's noise
    final = {"max": float(fres.max()), "min": float(fres.min()), "finite": bool(torch.isfinite(fres).all()),
             "noise_level": round(math.sqrt(w.n_steps * w.n_obs + w.n_nodes), 3)}
    log(f"batched f32: {ms_per_step:.1f} ms per batch of {R} -> {value:.1f} samples/min (|mean|={mean_norm:.4e}); "
        f"float64 final residuals {final['min']:.2f} .. {final['max']:.2f}")

    # roofline of the dominant kernels: each sweep = N_T step launches (+1 tiny sampling/init launch)
    fwd_avg_s = prof["fwd_ms"] / max(prof["fwd_sweeps"], 1) / w.n_steps / 1e3
    adj_avg_s = prof["adj_ms"] / max(prof["adj_sweeps"], 1) / w.n_steps / 1e3
    fb = step_bytes(info, 64, 4, "fwd")
    ab = step_bytes(info, 64, 4, "adj")
    fwd_gbs = fb / fwd_avg_s / 1e9
    adj_gbs = ab / adj_avg_s / 1e9
    # the a-priori estimate of the method's bytes per sweep-step of either direction, made before the
    # kernels were written (ball58, 64 float32 RHS, four state vectors: matrix 22.8 + rowptr 0.8 + B 1.1 +
    # dt/m 0.8 + state 199.8 + sensors 0.26 MB)
    survey_step_bytes = 225.5e6 if w.n_nodes == 195112 and R == 64 else None
    sweep_share = (prof["fwd_ms"] + prof["adj_ms"]) / (el * 1e3)
    log(f"forward step: {fwd_avg_s * 1e6:.2f} us, {fb / 1e6:.1f} MB -> {fwd_gbs:.0f} GB/s; transpose step: "
        f"{adj_avg_s * 1e6:.2f} us, {ab / 1e6:.1f} MB -> {adj_gbs:.0f} GB/s; sweeps = {100 * sweep_share:.1f}% of time")

    result = {
        "metric": "RTO samples/min at 2e5 DOF (batched FP32 sweeps, FP64 CGLS)",
        "value": round(value, 3), "unit": "samples/min", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: {w.n_nodes}-node mapped ball (P1 tets), variable c, absorbing boundary, "
                         f"{w.n_steps} leapfrog steps, {w.n_obs} sensors on r=0.9, {R} RTO samples x {n_iter} "
                         f"CGLS iterations with full reorthogonalisation as one 64-RHS block; float32 sweeps, "
                         f"float64 CGLS vectors/dots/scalars"),
            "n_nodes": w.n_nodes, "n_steps": w.n_steps, "n_obs": w.n_obs, "samples_per_step": R,
            "cgls_iters": n_iter, "rhs_block": 64, "cgls_dtype": "f64",
        },
        "roofline": roofline_record(fwd_avg_s, adj_avg_s, fb, ab, survey_step_bytes, sweep_share, w.name, 64),
        "final_residual_f64": final,
    }
    if not args.no_wide_probe:
        result["roofline"]["beyond_cache"] = wide_probe(pat, G, info, w, yobs, sigma, iters=args.wide_iters)

    if not args.no_plain:
        # plain float64 path: one sample at a time, float64 everywhere
        e1, x1 = eta[:1].contiguous(), xi[:1].contiguous()
        pat.rto_sample(G, yobs, e1, x1, sigma, w.prior_a, 2, sweep_prec="f64", rhs_block=1, stats=False)
        G.profile_enable(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        pat.rto_sample(G, yobs, e1, x1, sigma, w.prior_a, n_iter, sweep_prec="f64", rhs_block=1, stats=False)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        pprof = G.profile()
        G.profile_enable(False)
        plain = 60.0 / tp
        # the single-RHS step is the plain SpMV: its rate against the HBM peak, as for the batched step
        pf_s = pprof["fwd_ms"] / max(pprof["fwd_sweeps"], 1) / w.n_steps / 1e3
        pa_s = pprof["adj_ms"] / max(pprof["adj_sweeps"], 1) / w.n_steps / 1e3
        pfb, pab = step_bytes(info, 1, 8, "fwd"), step_bytes(info, 1, 8, "adj")
        result["plain_fp64"] = {"value": round(plain, 3), "unit": "samples/min", "rhs_block": 1,
                                "seconds_per_sample": round(tp, 3), "speedup_batched_f32": round(value / plain, 2),
                                "fwd_step": {"avg_launch_us": round(pf_s * 1e6, 3), "bytes_per_launch": pfb,
                                             "achieved_GBs": round(pfb / pf_s / 1e9, 1),
                                             "frac": round(pfb / pf_s / 1e9 / HBM_PEAK_GBS, 4)},
                                "adj_step": {"avg_launch_us": round(pa_s * 1e6, 3), "bytes_per_launch": pab,
                                             "achieved_GBs": round(pab / pa_s / 1e9, 1)},
                                "sweep_time_share": round((pprof["fwd_ms"] + pprof["adj_ms"]) / (tp * 1e3), 4)}
        log(f"plain f64 (1 sample, R=1): {tp:.2f} s -> {plain:.2f} samples/min; speed-up {value / plain:.1f}x; "
            f"forward step {pf_s * 1e6:.2f} us ({pfb / pf_s / 1e9:.0f} GB/s), transpose {pa_s * 1e6:.2f} us")

    if copy_probe:
        result["copy_probe"] = copy_probe
    if stream_probe:
        result["stream_probe"] = stream_probe
    if not args.no_uneven:
        names = tuple(args.uneven_set.split(","))
        result["uneven_batch"] = uneven_leg(pat, W, dev, n_iter, modes=args.uneven_modes, names=names)
    if args.lsqr:
        result["lsqr"] = lsqr_leg(pat, G, w, yobs, eta, xi, sigma, n_iter, R)
    if args.map:
        result["autograd_map"] = map_leg(G, w, dev, yobs, sigma)
    if args.wide:
        result["wide_block"] = wide_leg(pat, dev, G, info, w, yobs, sigma, n_iter)
    if args.spectral:
        result["spectral_prior"] = spectral_leg(pat, dev, G, w, yobs, sigma, n_iter)
    if args.big:
        result["ball100_single_sample"] = big_leg(pat, W, dev, n_iter)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(w, eta_h, xi_h, yobs.cpu().numpy(), sigma, n_iter, R)
        log(f"cpu baseline: {result['cpu_baseline']['value']:.4f} samples/min on "
            f"{result['cpu_baseline']['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
