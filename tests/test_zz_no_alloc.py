"""pat_forward_noalloc (the forward map with the library's fixed device scratch,
for callers that cannot allocate) against pat_forward.

Two calls in a row, the second with fewer right-hand sides, must each equal
pat_forward on the same input: bit for bit where both use the same RHS block
(small meshes), to the float64 / float32 parity bars of the forward map where
the scratch limits the block (the 195k-node ball).  A problem whose single
right-hand side does not fit the scratch is rejected before any device work.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


def _run_pair(G, dtype, Rs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for R in Rs:
        p0 = torch.as_tensor(rng.standard_normal((R, G.n_nodes)), dtype=dtype, device="cuda")
        y = torch.full((R, G.n_steps, G.n_obs), float("nan"), dtype=dtype, device="cuda")
        pat.pat_forward_noalloc(G, p0, y)
        ref = pat.pat_forward(G, p0)
        torch.cuda.synchronize()
        out.append((y, ref))
    return out


@pytest.mark.parametrize("dtype,Rs", [(torch.float64, (5, 2)), (torch.float32, (20, 3)), (torch.float64, (1, 1)),
                                      (torch.float32, (70, 9))])
def test_noalloc_equals_forward_small(dtype, Rs):
    w = W.make_workload("ball16")
    G = pat.Problem.from_workload(w)
    print(f"noalloc ball16 {dtype} R={Rs}", flush=True)
    for y, ref in _run_pair(G, dtype, Rs, 3):
        assert torch.isfinite(y).all()
        assert torch.equal(y, ref)


@pytest.mark.parametrize("dtype,Rs,tol", [(torch.float64, (6, 3), 1e-10), (torch.float32, (12, 5), 1e-4)])
def test_noalloc_equals_forward_fullsize(dtype, Rs, tol):
    """On the 195k-node ball one RHS block of pat_forward (8 or 16 RHS) does not fit the 64 MiB
    scratch, so the no-allocation path runs narrower blocks (other kernels, other summation
    order): equal to pat_forward within the parity bars of the forward map."""
    w = W.make_workload("ball58_fp64")
    G = pat.Problem.from_workload(w)
    print(f"noalloc ball58 {dtype} R={Rs}", flush=True)
    for y, ref in _run_pair(G, dtype, Rs, 4):
        assert torch.isfinite(y).all()
        err = float((y.double() - ref.double()).abs().max() / ref.double().abs().max())
        print(f"  rel max diff {err:.2e}")
        assert err < tol


def test_noalloc_rejects_oversized_problem():
    """A sensor at each of the 729 nodes over 12,000 steps: the data staging of one RHS alone
    (70 MB in float64) exceeds the 64 MiB scratch, so the call fails with PAT_ERR_INVALID_ARG
    and leaves y untouched."""
    w = W.make_workload("cube8_tiny")
    G = pat.Problem(w.coords, w.tets, None, False, w.dt, 12000, sensor_nodes=np.arange(w.n_nodes))
    p0 = torch.zeros((1, G.n_nodes), dtype=torch.float64, device="cuda")
    y = torch.full((1, G.n_steps, G.n_obs), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pat.PatError) as ei:
        pat.pat_forward_noalloc(G, p0, y)
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    assert "scratch" in str(ei.value)
    assert bool((y == 7.0).all())
    # float32: 35 MB of staging plus the state fit, so the same problem runs there
    p32 = torch.as_tensor(np.random.default_rng(5).standard_normal((1, G.n_nodes)), dtype=torch.float32,
                          device="cuda")
    y32 = torch.empty((1, G.n_steps, G.n_obs), dtype=torch.float32, device="cuda")
    pat.pat_forward_noalloc(G, p32, y32)
    assert torch.equal(y32, pat.pat_forward(G, p32))
