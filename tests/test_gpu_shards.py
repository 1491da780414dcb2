"""Sample sharding (how the sampler would spread over several GPUs): shards that draw
disjoint ranges of the same seed's streams (sample0) reproduce the single run.

* each shard's samples equal the matching rows of the single run bit for bit (the
  draws depend only on (seed, sample id), and with one RHS block size every sample's
  sweeps and solver arithmetic are the same wherever it sits in a block);
* the shards' (count, mean, M2) merged with Chan et al.'s pairwise formula equal the
  single run's mean and std to rounding.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


def _chan_merge(parts):
    """(n, mean, std with 1/(n-1)) per shard -> merged (n, mean, std)."""
    n, mean, m2 = 0, None, None
    for nb, mb, sb in parts:
        m2b = sb ** 2 * (nb - 1)
        if n == 0:
            n, mean, m2 = nb, mb.copy(), m2b
            continue
        d = mb - mean
        tot = n + nb
        mean = mean + d * (nb / tot)
        m2 = m2 + m2b + d * d * (n * nb / tot)
        n = tot
    return n, mean, np.sqrt(m2 / (n - 1))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_shards_reproduce_single_run(prec):
    w = W.make_workload("ball16")
    O = oracle.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    G = pat.Problem.from_workload(w)
    y = torch.as_tensor(yobs, device="cuda")
    kw = dict(sweep_prec=prec, rhs_block=8, seed=5)
    full = pat.rto_sample(G, y, None, None, sigma, w.prior_a, 10, n_samples=24, sample0=0, **kw)
    shards = [(0, 10), (10, 14)]
    parts = []
    for s0, cnt in shards:
        o = pat.rto_sample(G, y, None, None, sigma, w.prior_a, 10, n_samples=cnt, sample0=s0, **kw)
        assert torch.equal(o["samples"], full["samples"][s0:s0 + cnt]), (s0, cnt)
        parts.append((cnt, o["mean"].cpu().numpy(), o["std"].cpu().numpy()))
    n, mean, std = _chan_merge(parts)
    ref_m, ref_s = full["mean"].cpu().numpy(), full["std"].cpu().numpy()
    em = float(np.abs(mean - ref_m).max() / np.abs(ref_m).max())
    es = float(np.abs(std - ref_s).max() / np.abs(ref_s).max())
    print(f"{prec}: merged shards vs single run: mean {em:.1e}, std {es:.1e}")
    assert n == 24 and em < 1e-13 and es < 1e-12
