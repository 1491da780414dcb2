"""RHS blocks wider than 64: 128 and 256 right-hand sides per sweep.

A row of a float32 block of 256 RHS fills one wave (64 lanes x 16 bytes); 128
float32 RHS, or 128 float64 RHS, take half a wave or a whole one.  Checked:

* ball16: 130 samples (one ragged 256-block, or a full and a ragged 128-block)
  with float32 sweeps against the oracle on the same draws (1e-4 relative L2 on
  mean and std), and float64 sweeps with 128-blocks (1e-10 on the samples);
* blocks the step kernels cannot hold are rejected before any launch;
* the autotuner considers blocks beyond 64 only when S needs them;
* maximum sizes: on a 4.25M-node ball a 256-RHS float32 block exceeds the
  step kernels' 4 GiB state limit and is rejected; the tuner stops at 128;
* the merged multi-mesh step kernels with 128- and 256-RHS blocks equal the
  per-problem runs bit for bit.
The full-size check (ball58, the 64 stored oracle samples inside one 128- and
one 256-RHS block) is part of the stored-oracle test of test_gpu_fullsize.py.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ball16_130():
    w = W.make_workload("ball16")
    O = oracle.Problem.from_workload(w)
    G = pat.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    S, n_iter = 130, 10
    eta, xi = W.rto_draws(S, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
    ref, rres = O.rto(yobs, sigma, w.prior_a, n_iter, eta, xi)
    return w, G, (yobs, sigma, eta, xi, n_iter), ref, rres


@pytest.mark.parametrize("prec,rb,tol,solver", [("f32", 256, 1e-4, "cgls"), ("f32", 128, 1e-4, "cgls"),
                                              ("f64", 128, 1e-10, "cgls"), ("f64", 128, 1e-9, "lsqr")])
def test_wide_blocks_match_oracle(ball16_130, prec, rb, tol, solver):
    """Against the oracle's CGLS; LSQR has the same iterates in exact arithmetic (1e-9)."""
    w, G, (yobs, sigma, eta, xi, n_iter), ref, rres = ball16_130
    print(f"ball16 S=130 {prec} rhs_block={rb} {solver}", flush=True)
    out = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, n_iter, sweep_prec=prec,
                         rhs_block=rb, resid=True, solver=solver)
    rmean, rstd = oracle.stats(ref)
    em = _rel_l2(out["mean"].cpu().numpy(), rmean)
    es = _rel_l2(out["std"].cpu().numpy(), rstd)
    ex = _rel_l2(out["samples"].cpu().numpy(), ref)
    print(f"  mean {em:.2e} std {es:.2e} samples {ex:.2e}")
    assert em < tol and es < tol
    if prec == "f64":
        assert ex < tol
        assert float(np.abs(out["resid"].cpu().numpy() - rres).max() / np.abs(rres).max()) < tol


def test_wide_blocks_equal_narrow_sweeps(ball16_130):
    """One float64 iteration with 128-blocks and with 64-blocks: the sweeps compute each RHS the
    same way in any block; only the solver's dot products are summed in another order."""
    w, G, (yobs, sigma, eta, xi, _), ref, _ = ball16_130
    a = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, 1, sweep_prec="f64", rhs_block=128)
    b = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, 1, sweep_prec="f64", rhs_block=64)
    d = _rel_l2(a["samples"].cpu().numpy(), b["samples"].cpu().numpy())
    print(f"one iteration, 128- vs 64-blocks: {d:.2e}")
    assert d < 1e-14


def test_wide_block_errors(ball16_130):
    w, G, (yobs, sigma, eta, xi, n_iter), _, _ = ball16_130
    args = (G, _dev(yobs), _dev(eta[:3]), _dev(xi[:3]), sigma, w.prior_a, 2)
    for prec, rb in (("f64", 256), ("f32", 512), ("f32", 96)):
        with pytest.raises(pat.PatError) as ei:
            pat.rto_sample(*args, sweep_prec=prec, rhs_block=rb)
        assert ei.value.name == "PAT_ERR_INVALID_ARG"


def test_autotune_wide_candidates(ball16_130):
    w, G, _, _, _ = ball16_130
    before = G.info()["device_bytes"]
    rb, us = pat.autotune(G, 200, "f32")
    # the workspaces of the candidates not chosen are released again: the handle grows by at
    # most the chosen block's sweep state and staging, and a second identical call adds nothing
    def ws(b):  # sweep state (P, V, ping-pong) and the data staging of one block
        return 4 * w.n_nodes * b * 4 + w.n_steps * w.n_obs * b * 4

    grown = G.info()["device_bytes"] - before
    assert grown <= ws(rb), (grown, rb)
    after = G.info()["device_bytes"]
    rb2, _ = pat.autotune(G, 200, "f32")
    assert G.info()["device_bytes"] - after <= (0 if rb2 == rb else ws(rb2)), (rb, rb2)
    print(f"autotune ball16 S=200 f32: rb={rb}, {us:.1f} us per step pair")
    assert rb in (4, 8, 16, 32, 64, 128, 256) and us > 0
    rb64, _ = pat.autotune(G, 200, "f64")
    assert rb64 in (4, 8, 16, 32, 64, 128)
    rbs, _ = pat.autotune(G, 40, "f32")
    assert rbs <= 64


def test_block_state_limit_on_a_4m_node_mesh():
    """Maximum sizes: on a 4,251,528-node ball one 256-RHS float32 block's sweep state
    (N x 256 x 4 B = 4.35 GB) is beyond what the step kernels address, so an explicit
    rhs_block = 256 is rejected before any work; 128 runs; the autotuner asked for 256
    samples considers blocks up to 128 only."""
    X, T = W.ball_mesh(161)
    N = X.shape[0]
    assert N * 256 * 4 >= 1 << 32 > N * 128 * 4
    sensors = np.linspace(0, N - 1, 16).astype(np.int32)
    G = pat.Problem(X, T, None, True, 0.2 * 2.0 / 161, 4, sensor_nodes=sensors, check_dt=False)
    print(f"ball161: {N} nodes", flush=True)
    y = torch.zeros((4, 16), dtype=torch.float64, device="cuda")
    args = (G, y, None, None, 1.0, 0.01, 1)
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(*args, sweep_prec="f32", rhs_block=256, n_samples=2, seed=1)
    assert ei.value.name == "PAT_ERR_INVALID_ARG" and "4 GiB" in str(ei.value)
    out = pat.rto_sample(*args, sweep_prec="f32", rhs_block=128, n_samples=2, seed=1)
    assert torch.isfinite(out["samples"]).all()
    rb, us = pat.autotune(G, 256, "f32")
    print(f"autotune S=256 on {N} nodes: rhs_block {rb}", flush=True)
    assert rb <= 128 and us > 0


@pytest.mark.parametrize("rb", [128, 256])
def test_wide_block_merged_batch_equals_single(rb):
    """The merged multi-mesh step kernels with wide blocks: three small meshes in one
    batch (one merged launch per step) equal each mesh's own rto_sample bit for bit."""
    ws = [W.make_workload(n) for n in ("cube8_tiny", "ball16", "box12")]
    probs = [pat.Problem.from_workload(w) for w in ws]
    ys, sig = [], []
    for w in ws:
        O = oracle.Problem.from_workload(w)
        Y, yobs, sigma = oracle.synthesize(O, w)
        ys.append(_dev(yobs))
        sig.append(sigma)
    B = pat.Batch(probs)
    B.merge(1, 1)
    S = [rb // 2 + 3, rb - 5, 7]
    outs = pat.rto_sample_batch(B, ys, None, None, sig, 0.01, 4, sweep_prec="f32", rhs_block=rb, n_samples=S,
                                seed=[1, 2, 3])
    for m, (G, y, s) in enumerate(zip(probs, ys, sig)):
        ref = pat.rto_sample(G, y, None, None, s, 0.01, 4, sweep_prec="f32", rhs_block=rb, n_samples=S[m], seed=m + 1)
        assert torch.equal(outs[m]["samples"], ref["samples"]), (rb, m)
