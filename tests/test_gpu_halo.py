"""Halo-tile step kernels against the vector-lane kernels, bit for bit.

Float32 blocks of 64 RHS run on the halo-tile kernels; blocks of 32 run on the
vector-lane kernels.  Both sum each RHS column over the padded slots in the same
order with the same operations (Sec. 3 eq. (fully-discrete) row by row; the
transposed step of Sec. 5.1 eq. (adjoint-verlet)).  So the forward and transposed
maps of 64 columns equal those of the same columns in two blocks of 32, bit for
bit.  The meshes cover:
- a single partial tile (27 nodes);
- tiles split by the boundary-row budget;
- overflow rows (more than 16 entries) and sensor injections;
- the 195,112-node ball.
Parity of both paths with the oracle is in test_gpu_parity, test_gpu_fullsize and
test_gpu_tiny_meshes.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


@pytest.mark.parametrize("name", ["cube8_tiny", "ball16", "box12", "ball58_batched"])
def test_halo_equals_vector_lanes(name):
    w = W.make_workload(name)
    G = pat.Problem.from_workload(w)
    rng = np.random.default_rng(61)
    P = torch.as_tensor(rng.standard_normal((64, w.n_nodes)), dtype=torch.float32, device="cuda")
    YH = torch.as_tensor(rng.standard_normal((64, w.n_steps, w.n_obs)), dtype=torch.float32, device="cuda")
    print(f"{name}: forward", flush=True)
    y64 = pat.pat_forward(G, P)
    y32 = torch.cat([pat.pat_forward(G, P[:32].contiguous()), pat.pat_forward(G, P[32:].contiguous())])
    assert torch.equal(y64, y32)
    print(f"{name}: transpose", flush=True)
    a64 = pat.pat_adjoint(G, YH)
    a32 = torch.cat([pat.pat_adjoint(G, YH[:32].contiguous()), pat.pat_adjoint(G, YH[32:].contiguous())])
    assert torch.equal(a64, a32)
    assert torch.isfinite(y64).all() and torch.isfinite(a64).all()
