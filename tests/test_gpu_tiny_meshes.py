"""Tiny meshes against the oracle: the launch mapping at its edges.

Balls of 2, 3 and 5 cells per axis (27, 64 and 216 nodes) give fewer row tiles
than there are XCDs, partial tiles and partial waves; 3 sensors leave most waves
without an injected row, 40 sensors put one in nearly every wave.  The forward
and transpose maps (Stormer-Verlet, Sec. 3; its transpose, Sec. 5.1)
are checked against the oracle at 1, 2, 5 and 64 RHS in float64 (1e-11 of the
largest output, rounding only) and float32 (2e-5), and the two GPU maps against
each other through the discrete transpose identity.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")

CASES = {}


def _case(n, n_sens):
    key = (n, n_sens)
    if key not in CASES:
        coords, tets = W.ball_mesh(n)
        w = W.Workload(name=f"ball{n}_s{n_sens}", coords=coords, tets=tets, c_tet=None, absorbing=True,
                       dt=0.2 * 2 / n, n_steps=12, sensor_pos=W.fibonacci_sphere(n_sens, 0.7),
                       p0_true=W.smooth_bump(coords, 0.8))
        CASES[key] = (w, oracle.Problem.from_workload(w), pat.Problem.from_workload(w))
    return CASES[key]


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("R", [1, 2, 5, 64])
@pytest.mark.parametrize("n_sens", [3, 40])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_tiny_forward_adjoint(n, n_sens, R):
    w, O, G = _case(n, n_sens)
    rng = np.random.default_rng(1000 * n + 10 * n_sens + R)
    p0 = rng.standard_normal((R, w.n_nodes))
    yh = rng.standard_normal((R, w.n_steps, w.n_obs))
    print(f"tiny ball n={n} N={w.n_nodes} sensors={n_sens} R={R}", flush=True)
    y64 = pat.pat_forward(G, _dev(p0)).cpu().numpy()
    a64 = pat.pat_adjoint(G, _dev(yh)).cpu().numpy()
    assert _rel_max(y64, O.forward(p0)) < 1e-11
    assert _rel_max(a64, O.adjoint(yh)) < 1e-11
    p32, yh32 = p0.astype(np.float32), yh.astype(np.float32)
    y32 = pat.pat_forward(G, _dev(p32, torch.float32)).cpu().numpy().astype(np.float64)
    a32 = pat.pat_adjoint(G, _dev(yh32, torch.float32)).cpu().numpy().astype(np.float64)
    assert _rel_max(y32, O.forward(p32.astype(np.float64))) < 2e-5
    assert _rel_max(a32, O.adjoint(yh32.astype(np.float64))) < 2e-5
    # <G p, yh> = <p, G^T yh>, both sides from the GPU maps
    lhs = np.einsum("rts,rts->r", y64, yh)
    rhs = np.einsum("rn,rn->r", p0, a64)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * np.linalg.norm(y64.reshape(R, -1), axis=1)
                  * np.linalg.norm(yh.reshape(R, -1), axis=1))


@pytest.mark.parametrize("n", [2, 5])
def test_tiny_rto_single_rhs(n):
    """A few single-RHS RTO solves (float64 sweeps, the plain path) on a tiny mesh."""
    w, O, G = _case(n, 40)
    rng = np.random.default_rng(50 + n)
    yobs = O.forward(w.p0_true[None])[0] + 0.01 * rng.standard_normal((w.n_steps, w.n_obs))
    S, n_iter, sigma = 3, 8, 0.05
    eta = rng.standard_normal((S, w.n_steps, w.n_obs))
    xi = rng.standard_normal((S, w.n_nodes))
    ref, res = O.rto(yobs, sigma, w.prior_a, n_iter, eta, xi)
    out = pat.rto_sample(G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, n_iter, sweep_prec="f64",
                         rhs_block=1, resid=True)
    got = out["samples"].cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10
    assert _rel_max(out["resid"].cpu().numpy(), res) < 1e-10
