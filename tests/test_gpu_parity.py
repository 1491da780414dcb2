"""GPU parity: libpat (HIP, through the C ABI) against the CPU FP64 oracle.

Small problems, where the oracle runs in seconds, spanning several tiles, ragged
RHS counts and both precisions.  Tolerances:
  * float64 sweeps: the kernels evaluate the three-level form of the step with FMA
    contraction, the oracle the literal three substeps without; both are exact
    in exact arithmetic, so differences are rounding only (bound 1e-11 relative
    to the largest output over <= 1000 steps).
  * float32 sweeps: unit roundoff 6e-8 per operation over N_T steps; the bound
    below is 2e-5 relative to the largest output.
  * RTO: float64 path 1e-10 relative L2 on samples, mean and std; float32
    sweeps with float64 CGLS 1e-4 relative L2 on mean and std.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


def _rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {}


def _case(name, n_steps=None):
    key = (name, n_steps)
    if key not in CASES:
        w = W.make_workload(name)
        if n_steps is not None:
            w.n_steps = n_steps
        CASES[key] = (w, oracle.Problem.from_workload(w), pat.Problem.from_workload(w))
    return CASES[key]


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("name,R", [("cube8_tiny", 1), ("cube8_tiny", 3), ("cube8_tiny", 10), ("ball16", 1),
                                    ("ball16", 5), ("ball16", 64), ("ball16", 70)])
def test_forward_f64(name, R):
    w, O, G = _case(name)
    p0 = np.random.default_rng(R).standard_normal((R, w.n_nodes))
    ref = O.forward(p0)
    got = pat.pat_forward(G, _dev(p0)).cpu().numpy()
    assert got.shape == ref.shape
    assert _rel_max(got, ref) < 1e-11


@pytest.mark.parametrize("name,R", [("cube8_tiny", 1), ("cube8_tiny", 10), ("ball16", 2), ("ball16", 64),
                                    ("ball16", 65)])
def test_adjoint_f64(name, R):
    w, O, G = _case(name)
    yh = np.random.default_rng(100 + R).standard_normal((R, w.n_steps, w.n_obs))
    ref = O.adjoint(yh)
    got = pat.pat_adjoint(G, _dev(yh)).cpu().numpy()
    assert _rel_max(got, ref) < 1e-11


@pytest.mark.parametrize("name,R", [("cube8_tiny", 4), ("ball16", 16), ("ball16", 64)])
def test_forward_adjoint_f32(name, R):
    w, O, G = _case(name)
    rng = np.random.default_rng(7)
    p0 = rng.standard_normal((R, w.n_nodes))
    yh = rng.standard_normal((R, w.n_steps, w.n_obs))
    y32 = pat.pat_forward(G, _dev(p0, torch.float32)).cpu().numpy()
    a32 = pat.pat_adjoint(G, _dev(yh, torch.float32)).cpu().numpy()
    assert y32.dtype == np.float32
    assert _rel_max(y32.astype(np.float64), O.forward(p0.astype(np.float32).astype(np.float64))) < 2e-5
    assert _rel_max(a32.astype(np.float64), O.adjoint(yh.astype(np.float32).astype(np.float64))) < 2e-5


@pytest.mark.parametrize("name", ["cube8_tiny", "ball16"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_transpose_identity_gpu(name, dtype):
    """<G p, yhat> = <p, G^T yhat> with both maps on the GPU (Sec. 6.1 discrete adjoint test)."""
    w, O, G = _case(name)
    rng = np.random.default_rng(4)
    R = 3
    p = rng.standard_normal((R, w.n_nodes))
    yh = rng.standard_normal((R, w.n_steps, w.n_obs))
    y = pat.pat_forward(G, _dev(p, dtype)).cpu().numpy().astype(np.float64)
    a = pat.pat_adjoint(G, _dev(yh, dtype)).cpu().numpy().astype(np.float64)
    p64 = _dev(p, dtype).cpu().numpy().astype(np.float64)
    yh64 = _dev(yh, dtype).cpu().numpy().astype(np.float64)
    lhs = np.einsum("rts,rts->r", y, yh64)
    rhs = np.einsum("rn,rn->r", p64, a)
    tol = 1e-13 if dtype == torch.float64 else 2e-5
    assert np.all(np.abs(lhs - rhs) <= tol * np.abs(lhs)), (lhs, rhs)


def _rto_inputs(w, O, S=None, n_iter=None):
    Y, yobs, sigma = oracle.synthesize(O, w)
    S = w.n_samples if S is None else S
    eta, xi = W.rto_draws(S, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
    return yobs, sigma, eta, xi, (w.n_iter if n_iter is None else n_iter)


@pytest.mark.parametrize("name,S,rb", [("cube8_tiny", 10, 0), ("ball16", 16, 0), ("ball16", 16, 4),
                                       ("ball16", 5, 1)])
def test_rto_f64_matches_oracle(name, S, rb):
    w, O, G = _case(name)
    yobs, sigma, eta, xi, n_iter = _rto_inputs(w, O, S)
    ref, rres = O.rto(yobs, sigma, w.prior_a, n_iter, eta, xi)
    rmean, rstd = oracle.stats(ref)
    out = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, n_iter, sweep_prec="f64",
                         rhs_block=rb, resid=True)
    got = out["samples"].cpu().numpy()
    assert _rel_l2(got, ref) < 1e-10
    assert _rel_l2(out["mean"].cpu().numpy(), rmean) < 1e-10
    assert _rel_l2(out["std"].cpu().numpy(), rstd) < 1e-10
    assert _rel_max(out["resid"].cpu().numpy(), rres) < 1e-10


@pytest.mark.parametrize("name,S", [("cube8_tiny", 10), ("ball16", 64)])
def test_rto_f32_sweeps_match_oracle(name, S):
    w, O, G = _case(name)
    yobs, sigma, eta, xi, n_iter = _rto_inputs(w, O, S)
    ref, _ = O.rto(yobs, sigma, w.prior_a, n_iter, eta, xi)
    rmean, rstd = oracle.stats(ref)
    out = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, n_iter, sweep_prec="f32")
    em = _rel_l2(out["mean"].cpu().numpy(), rmean)
    es = _rel_l2(out["std"].cpu().numpy(), rstd)
    print(f"{name}: f32 sweeps mean rel L2 {em:.3e}, std rel L2 {es:.3e}")
    assert em < 1e-4 and es < 1e-4


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_rto_iid_prior_matches_oracle(prec, tol):
    """a = 0: the paper's independent prior with precision M_L, L = M_L^{1/2} (Sec. 4.1.1 eq. (iid-prior))."""
    w, O, G = _case("ball16")
    yobs, sigma, eta, xi, n_iter = _rto_inputs(w, O, 12)
    ref, rres = O.rto(yobs, sigma, 0.0, n_iter, eta, xi)
    rmean, rstd = oracle.stats(ref)
    out = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, 0.0, n_iter, sweep_prec=prec, resid=True)
    em = _rel_l2(out["mean"].cpu().numpy(), rmean)
    es = _rel_l2(out["std"].cpu().numpy(), rstd)
    print(f"a = 0, {prec} sweeps: mean rel L2 {em:.3e}, std rel L2 {es:.3e}")
    assert em < tol and es < tol
    if prec == "f64":
        assert _rel_l2(out["samples"].cpu().numpy(), ref) < tol
        assert _rel_max(out["resid"].cpu().numpy(), rres) < tol


def test_rto_edge_cases():
    """One iteration, one sample (no std), no reorthogonalisation."""
    w, O, G = _case("ball16")
    yobs, sigma, eta, xi, _ = _rto_inputs(w, O, 3)
    for n_iter, reorth, S in ((1, True, 1), (3, False, 3), (2, True, 3)):
        ref, _ = O.rto(yobs, sigma, w.prior_a, n_iter, eta[:S], xi[:S], reorth=reorth)
        out = pat.rto_sample(G, _dev(yobs), _dev(eta[:S]), _dev(xi[:S]), sigma, w.prior_a, n_iter,
                             reorth=reorth, stats=S > 1)
        assert _rel_l2(out["samples"].cpu().numpy(), ref) < 1e-11


def test_runtime_errors():
    w, O, G = _case("cube8_tiny")
    p0 = _dev(np.zeros((2, w.n_nodes)))
    with pytest.raises(ValueError):
        pat.pat_forward(G, p0[:, :-1].contiguous())
    yobs = _dev(np.zeros((w.n_steps, w.n_obs)))
    eta = _dev(np.zeros((2, w.n_steps, w.n_obs)))
    xi = _dev(np.zeros((2, w.n_nodes)))
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(G, yobs, eta, xi, -1.0, 0.01, 5)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(pat.PatError):
        pat.rto_sample(G, yobs, eta, xi, 1.0, 0.01, 5, rhs_block=3)
    bad = _dev(np.full((w.n_steps, w.n_obs), np.nan))
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(G, bad, eta, xi, 1.0, 0.01, 2)
    assert ei.value.name == "PAT_ERR_NONFINITE"
    # empty inputs: no right-hand sides, no samples, no iterations
    with pytest.raises(pat.PatError) as ei:
        pat.pat_forward(G, _dev(np.zeros((0, w.n_nodes))))
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(pat.PatError) as ei:
        pat.pat_adjoint(G, _dev(np.zeros((0, w.n_steps, w.n_obs))))
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(G, yobs, None, None, 1.0, 0.01, 2, n_samples=0, stats=False)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(G, yobs, eta, xi, 1.0, 0.01, 0)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"


def test_binding_works_when_torch_is_not_imported_first():
    """A fresh process that creates a problem before importing torch itself, then makes
    calls that need torch's stream (regression: torch failed to find the GPU when libpat
    had initialised HIP first)."""
    import os
    import subprocess
    import sys
    code = ("import workloads as W\n"
            "from paper_2607_21373_amd import pat\n"
            "G = pat.Problem.from_workload(W.make_workload('cube8_tiny'))\n"
            "rb, us = pat.autotune(G, 8, 'f32')\n"
            "print('ok', rb)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    print(r.stdout[-500:], r.stderr[-2000:])
    assert r.returncode == 0 and "ok" in r.stdout
