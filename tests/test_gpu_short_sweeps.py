"""Sweeps of 1 to 4 steps against the oracle: the start and the end of the three-level recurrences.

The step kernels carry one state vector per direction and rotate three buffers (Sec. 3
eq. (fully-discrete); Sec. 5.1 eqs. (backward-recursion), (adjoint-verlet)).  Short sweeps put every
launch of a sweep next to its start or its end: the forward's first step (S^{-1} = S^0 = p^0), the
final sampling-only launch, the transposed sweep's start values (q_{-1} = 0, q_0 = (dt/2m) Pi^T yhat^{N_T}),
its closing launch (with N_T = 1 it follows the start directly) and the placement of the result in the
buffer rotation.  Each block width runs its own kernel family: one float64 RHS (scalar lanes), 16 float64
RHS (vector lanes), 2 float32 RHS (scalar lanes) and 64 float32 RHS (halo tiles).  Bars: float64 1e-11
of the largest output (rounding only), float32 2e-5.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")

_CACHE = {}


def _problems(n_steps):
    if n_steps not in _CACHE:
        w = W.make_workload("ball16")
        _CACHE[n_steps] = (w, oracle.Problem.from_workload(w, n_steps=n_steps),
                           pat.Problem.from_workload(w, n_steps=n_steps))
    return _CACHE[n_steps]


def _rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n_steps", [1, 2, 3, 4])
@pytest.mark.parametrize("R,dtype,tol", [(1, torch.float64, 1e-11), (16, torch.float64, 1e-11),
                                         (2, torch.float32, 2e-5), (64, torch.float32, 2e-5)])
def test_short_sweeps(n_steps, R, dtype, tol):
    w, O, G = _problems(n_steps)
    print(f"short sweep N_T={n_steps} R={R} {dtype}", flush=True)
    rng = np.random.default_rng(100 + 7 * n_steps + R)
    x = rng.standard_normal((R, w.n_nodes))
    yh = rng.standard_normal((R, n_steps, O.n_obs))
    y = pat.pat_forward(G, torch.as_tensor(x, dtype=dtype, device="cuda")).double().cpu().numpy()
    a = pat.pat_adjoint(G, torch.as_tensor(yh, dtype=dtype, device="cuda")).double().cpu().numpy()
    torch.cuda.synchronize()
    assert _rel_max(y, O.forward(x)) < tol
    assert _rel_max(a, O.adjoint(yh)) < tol
