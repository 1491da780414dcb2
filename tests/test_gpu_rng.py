"""The sampler's own perturbations: device Philox4x64-10 + Box-Muller against the oracle.

* pat_draw_normals equals the oracle's generator for both kinds, several seeds,
  stream offsets and ragged lengths (the cipher words are integers and must
  agree exactly; the transform then differs only by the rounding of log, cos
  and sin: 1e-13 relative, 1e-14 absolute);
* rto_sample with eta = xi = NULL equals rto_sample fed the same streams, and the
  oracle's RTO fed the oracle's draws (1e-10, float64 sweeps);
* argument errors.
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


@pytest.mark.parametrize("seed,kind,k0,S,length", [(0, 0, 0, 3, 1), (1, 0, 0, 5, 1001), (2**63 + 5, 1, 7, 4, 37),
                                                   (12345, 1, 0, 2, 4), (99, 0, 1 << 40, 2, 4099)])
def test_draw_normals_match_oracle(seed, kind, k0, S, length):
    print(f"draw seed={seed} kind={kind} k0={k0} S={S} len={length}", flush=True)
    got = pat.draw_normals(seed, kind, k0, S, length).cpu().numpy()
    ref = oracle.normals(seed, kind, k0, S, length)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_draw_normals_large_moments():
    z = pat.draw_normals(2024, 0, 0, 8, 1 << 20)
    m, v = float(z.mean()), float(z.var())
    assert abs(m) < 5 / np.sqrt(z.numel()) and abs(v - 1) < 5 * np.sqrt(2 / z.numel())
    ref = oracle.normals(2024, 0, 5, 1, 1 << 20)[0]
    np.testing.assert_allclose(z[5].cpu().numpy(), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name,S,rb,solver", [("cube8_tiny", 10, 0, "cgls"), ("ball16", 6, 4, "lsqr")])
def test_rto_device_draws(name, S, rb, solver):
    w = W.make_workload(name)
    O = oracle.Problem.from_workload(w)
    G = pat.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    seed, k0 = 31, 3
    M = w.n_steps * w.n_obs
    eta = oracle.normals(seed, 0, k0, S, M).reshape(S, w.n_steps, w.n_obs)
    xi = oracle.normals(seed, 1, k0, S, w.n_nodes)
    ref, _ = O.rto(yobs, sigma, w.prior_a, w.n_iter, eta, xi, solver=solver)
    a = pat.rto_sample(G, _dev(yobs), None, None, sigma, w.prior_a, w.n_iter, rhs_block=rb, solver=solver,
                       n_samples=S, seed=seed, sample0=k0)
    b = pat.rto_sample(G, _dev(yobs), pat.draw_normals(seed, 0, k0, S, M).reshape(S, w.n_steps, w.n_obs),
                       pat.draw_normals(seed, 1, k0, S, w.n_nodes), sigma, w.prior_a, w.n_iter, rhs_block=rb,
                       solver=solver)
    sa, sb = a["samples"].cpu().numpy(), b["samples"].cpu().numpy()
    np.testing.assert_array_equal(sa, sb)
    err = float(np.linalg.norm(sa - ref) / np.linalg.norm(ref))
    print(f"{name} device-drawn RTO vs oracle: {err:.2e}")
    assert err < 1e-10


def test_rng_argument_errors():
    w = W.make_workload("cube8_tiny")
    G = pat.Problem.from_workload(w)
    y = _dev(np.zeros((w.n_steps, w.n_obs)))
    with pytest.raises(pat.PatError) as ei:
        pat.draw_normals(0, 2, 0, 1, 4)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(ValueError):
        pat.rto_sample(G, y, None, _dev(np.zeros((2, w.n_nodes))), 1.0, 0.01, 2)
    with pytest.raises(pat.PatError) as ei:
        pat.rto_sample(G, y, None, None, 1.0, 0.01, 2, n_samples=2, sample0=-1)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    assert pat.draw_normals(0, 0, 0, 0, 5).shape == (0, 5)
