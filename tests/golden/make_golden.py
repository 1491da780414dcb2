"""Write the stored expected values for the full-size 2e5-node ball problem.

Runs the CPU FP64 oracle only (``oracle/``) on the seeded inputs of
``workloads`` and stores posterior mean and standard deviation (eq. (ergodic))
of the RTO samples (Algorithm 1, CGLS with full reorthogonalisation, 100
iterations), plus checksums of the synthetic data so that a consumer can
confirm it regenerated the same inputs.

    python tests/golden/make_golden.py ball58_fp64       # 16 samples  (~40 min, 8 cores)
    python tests/golden/make_golden.py ball58_batched    # 64 samples  (~3 h, 8 cores)
    python tests/golden/make_golden.py ball100_forward   # forward map on the 10^6-node ball (~2 min)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def main(name):
    w = W.make_workload(name)
    log(f"{name}: N={w.n_nodes} E={w.tets.shape[0]} N_T={w.n_steps} N_obs={w.n_obs} S={w.n_samples} "
        f"iters={w.n_iter} threads={oracle.num_threads()}")
    P = oracle.Problem.from_workload(w)
    # stability sanity check: a random initial state must not grow over the whole window
    x = np.random.default_rng(11).standard_normal(w.n_nodes)
    yr = P.forward(x)
    assert np.isfinite(yr).all() and np.abs(yr[-50:]).max() < 10 * np.abs(yr[:50]).max(), "unstable dt"
    Y, yobs, sigma = oracle.synthesize(P, w)
    log(f"data: max|Y|={np.abs(Y).max():.6e} sigma={sigma:.6e}")
    eta, xi = W.rto_draws(w.n_samples, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
    t0 = time.time()
    samples, resid = P.rto(yobs, sigma, w.prior_a, w.n_iter, eta, xi, reorth=True)
    el = time.time() - t0
    mean, std = oracle.stats(samples)
    log(f"rto done in {el:.1f} s; |mean|={np.linalg.norm(mean):.6e} |std|={np.linalg.norm(std):.6e}")
    out = os.path.join(HERE, f"{name}_rto.npz")
    np.savez_compressed(
        out, mean=mean, std=std, sigma=sigma, resid=resid,
        yobs_sum=yobs.sum(), yobs_norm=np.linalg.norm(yobs), sample_norms=np.linalg.norm(samples, axis=1),
        sample0=samples[0])
    meta = {"workload": name, "n_nodes": w.n_nodes, "n_steps": w.n_steps, "n_obs": w.n_obs,
            "n_samples": w.n_samples, "n_iter": w.n_iter, "prior_a": w.prior_a, "rto_seed": w.rto_seed,
            "noise_seed": w.noise_seed, "sigma": sigma, "oracle_seconds": el,
            "oracle_threads": oracle.num_threads(),
            "command": f"python tests/golden/make_golden.py {name}"}
    with open(os.path.join(HERE, f"{name}_rto.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {out}")


# sensors whose traces the 10^6-node forward map stores: every 128th of the 1024
BALL100_SENSORS = tuple(range(0, 1024, 128))


def ball100_forward():
    """Forward map Y = G p0 (Sec. 3 eq. (discrete-wave-matrix)) of the inclusion phantom on the
    10^6-node ball, traces of BALL100_SENSORS over all 1000 steps."""
    w = W.make_workload("ball100")
    log(f"ball100: N={w.n_nodes} E={w.tets.shape[0]} N_T={w.n_steps} N_obs={w.n_obs} threads={oracle.num_threads()}")
    P = oracle.Problem.from_workload(w)
    t0 = time.time()
    Y = P.forward(w.p0_true)
    el = time.time() - t0
    sens = np.array(BALL100_SENSORS)
    out = os.path.join(HERE, "ball100_forward.npz")
    np.savez_compressed(out, sensors=sens, traces=Y[:, sens], y_max=np.abs(Y).max(), y_norm=np.linalg.norm(Y),
                        p0_sum=w.p0_true.sum(), p0_norm=np.linalg.norm(w.p0_true))
    meta = {"workload": "ball100", "n_nodes": w.n_nodes, "n_steps": w.n_steps, "n_obs": w.n_obs,
            "sensors": list(BALL100_SENSORS), "oracle_seconds": el, "oracle_threads": oracle.num_threads(),
            "command": "python tests/golden/make_golden.py ball100_forward"}
    with open(os.path.join(HERE, "ball100_forward.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {out} (forward map {el:.1f} s)")


if __name__ == "__main__":
    for n in sys.argv[1:]:
        ball100_forward() if n == "ball100_forward" else main(n)
