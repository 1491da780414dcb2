"""Uneven multi-mesh batch (one merged launch per time step) and the RHS-block autotuner.

* rto_sample_batch equals rto_sample on each problem alone, bit for bit: the
  merged launch runs the same per-row arithmetic (float32 and float64 sweeps,
  CGLS and LSQR, a vector-lane block that merges the meshes and a scalar-lane
  block that launches them one after another within each step);
* against the oracle on small meshes (float64: 1e-10);
* unequal sample counts spanning several RHS blocks;
* the three launch modes of the batch give identical results;
* the autotuner returns a valid block and rto_sample(rhs_block=0) then uses it;
* argument errors;
* the three full-size meshes (40^3 cube, 60^3 ball, 120x120x30 slab, 512
  sensors each, 1000 steps): forward sweeps sampled against the oracle and a
  short batched solve equal to the per-mesh solves.
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


@pytest.fixture(scope="module")
def small():
    ws = [W.make_workload("cube8_tiny"), W.make_workload("ball16"), W.make_workload("box12")]
    cases = []
    for w in ws:
        O = oracle.Problem.from_workload(w)
        G = pat.Problem.from_workload(w)
        Y, yobs, sigma = oracle.synthesize(O, w)
        cases.append((w, O, G, yobs, sigma))
    return cases


def _inputs(cases, S):
    out = []
    for (w, O, G, yobs, sigma), s in zip(cases, S):
        eta, xi = W.rto_draws(s, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
        out.append((_dev(yobs), _dev(eta), _dev(xi), sigma))
    return out


@pytest.mark.parametrize("prec,rb,solver", [("f32", 16, "cgls"), ("f64", 8, "lsqr"), ("f32", 2, "cgls"),
                                            ("f64", 16, "cgls")])
def test_batch_equals_single(small, prec, rb, solver):
    S = (10, 12, 7)
    inp = _inputs(small, S)
    B = pat.Batch([c[2] for c in small])
    n_iter = 20
    print(f"batch prec={prec} rb={rb} solver={solver}", flush=True)
    outs = pat.rto_sample_batch(B, [i[0] for i in inp], [i[1] for i in inp], [i[2] for i in inp],
                                [i[3] for i in inp], [c[0].prior_a for c in small], n_iter, sweep_prec=prec,
                                rhs_block=rb, solver=solver, resid=True, diag=True)
    for (w, O, G, yobs, sigma), (y, eta, xi, sg), o in zip(small, inp, outs):
        ref = pat.rto_sample(G, y, eta, xi, sg, w.prior_a, n_iter, sweep_prec=prec, rhs_block=rb, solver=solver,
                             resid=True, diag=True)
        for k in ("samples", "mean", "std", "resid", "diag"):
            assert torch.equal(o[k], ref[k]), (w.name, k)


@pytest.mark.parametrize("mf,ma", [(0, 0), (1, 1), (2, 2), (2, 1), (0, 2)])
def test_batch_launch_modes_agree(small, mf, ma):
    """Merged per step, one launch per problem per step, whole sweeps per problem: identical results."""
    S = (6, 9, 4)
    inp = _inputs(small, S)
    B = pat.Batch([c[2] for c in small])
    args = ([i[0] for i in inp], [i[1] for i in inp], [i[2] for i in inp], [i[3] for i in inp],
            [c[0].prior_a for c in small], 12)
    B.merge(1, 1)
    ref = pat.rto_sample_batch(B, *args, sweep_prec="f32", rhs_block=16)
    B.merge(mf, ma)
    out = pat.rto_sample_batch(B, *args, sweep_prec="f32", rhs_block=16)
    for a, b in zip(out, ref):
        assert torch.equal(a["samples"], b["samples"])
    with pytest.raises(pat.PatError):
        B.merge(3, 0)


def test_batch_mixed_priors(small):
    """One problem with the spectral prior (latent-space solve), the others with the FE factor."""
    G1 = small[1][2]
    pat.spectral_prior_set(G1, 8, -1.25, 2.5, 0.3, 3.0)
    try:
        B = pat.Batch([c[2] for c in small])
        ys = [_dev(c[3]) for c in small]
        prior, S = ["fe", "spectral", "fe"], [4, 6, 5]
        outs = pat.rto_sample_batch(B, ys, None, None, [c[4] for c in small], 0.01, 10, sweep_prec="f32",
                                    rhs_block=8, n_samples=S, seed=[1, 2, 3], prior=prior)
        for m, c in enumerate(small):
            ref = pat.rto_sample(c[2], ys[m], None, None, c[4], 0.01, 10, sweep_prec="f32", rhs_block=8,
                                 n_samples=S[m], seed=m + 1, prior=prior[m])
            assert torch.equal(outs[m]["samples"], ref["samples"]), m
    finally:
        pat.spectral_prior_set(G1, None, 0, 0, 0, 0)


def test_batch_matches_oracle(small):
    S = (10, 16, 6)
    inp = _inputs(small, S)
    B = pat.Batch([c[2] for c in small])
    outs = pat.rto_sample_batch(B, [i[0] for i in inp], [i[1] for i in inp], [i[2] for i in inp],
                                [i[3] for i in inp], [c[0].prior_a for c in small], 25, sweep_prec="f64",
                                rhs_block=16)
    for (w, O, G, yobs, sigma), (y, eta, xi, sg), o in zip(small, inp, outs):
        ref, _ = O.rto(yobs, sigma, w.prior_a, 25, eta.cpu().numpy(), xi.cpu().numpy())
        err = float(np.linalg.norm(o["samples"].cpu().numpy() - ref) / np.linalg.norm(ref))
        print(f"{w.name}: batch f64 vs oracle {err:.2e}")
        assert err < 1e-10


def test_batch_unequal_blocks_and_device_draws(small):
    """S = 5, 19, 9 with 8-RHS blocks: three blocks for the second mesh, zero RHS for the others."""
    B = pat.Batch([c[2] for c in small])
    ys = [_dev(c[3]) for c in small]
    outs = pat.rto_sample_batch(B, ys, None, None, [c[4] for c in small], 0.01, 15, sweep_prec="f32", rhs_block=8,
                                n_samples=[5, 19, 9], seed=[3, 4, 5], sample0=[0, 7, 2])
    for (w, O, G, yobs, sigma), y, o, S, sd, s0 in zip(small, ys, outs, (5, 19, 9), (3, 4, 5), (0, 7, 2)):
        ref = pat.rto_sample(G, y, None, None, sigma, 0.01, 15, sweep_prec="f32", rhs_block=8, n_samples=S,
                             seed=sd, sample0=s0)
        assert torch.equal(o["samples"], ref["samples"]) and torch.equal(o["std"], ref["std"])


def test_autotune(small):
    w, O, G, yobs, sigma = small[1]
    rb, us = pat.autotune(G, 12, "f32")
    print(f"autotune ball16 S=12: rb={rb} priced {us:.1f} us/step")
    assert rb in (1, 2, 4, 8, 16) and us > 0
    eta, xi = W.rto_draws(12, w.n_steps, w.n_obs, w.n_nodes, 9)
    args = (G, _dev(yobs), _dev(eta), _dev(xi), sigma, w.prior_a, 10)
    a = pat.rto_sample(*args, sweep_prec="f32", rhs_block=0)
    b = pat.rto_sample(*args, sweep_prec="f32", rhs_block=rb)
    assert torch.equal(a["samples"], b["samples"])
    B = pat.Batch([c[2] for c in small])
    rbb, usb = B.autotune(16, "f32")
    assert rbb in (1, 2, 4, 8, 16) and usb > 0


def test_batch_errors(small):
    w2 = W.make_workload("ball16")
    w2.n_steps = 150
    G2 = pat.Problem.from_workload(w2)
    with pytest.raises(pat.PatError) as ei:
        pat.Batch([small[0][2], G2])
    assert ei.value.name == "PAT_ERR_INVALID_ARG"
    with pytest.raises(pat.PatError):
        pat.Batch([small[0][2], small[0][2]])
    with pytest.raises(pat.PatError):
        pat.Batch([small[0][2]] * 5)
    B = pat.Batch([c[2] for c in small])
    inp = _inputs(small, (2, 2, 2))
    prms = (pat.RtoParams * 3)()
    with pytest.raises(pat.PatError) as ei:
        # per-problem n_iter differs: rejected before any launch
        import ctypes
        S = (ctypes.c_int64 * 3)(2, 2, 2)
        ys, smp = [(ctypes.c_void_p * 3)() for _ in range(2)]
        keep = []
        for m, (c, i) in enumerate(zip(small, inp)):
            prms[m].sigma, prms[m].prior_a, prms[m].n_iter, prms[m].reorth = i[3], 0.01, 3 + m, 1
            prms[m].eta, prms[m].xi = i[1].data_ptr(), i[2].data_ptr()
            out = torch.empty((2, c[0].n_nodes), dtype=torch.float64, device="cuda")
            keep.append(out)
            ys[m], smp[m] = i[0].data_ptr(), out.data_ptr()
        pat._check(pat.load().rto_sample_batch(B._h, ys, prms, S, smp, None, None, None, None))
    assert ei.value.name == "PAT_ERR_INVALID_ARG"


@pytest.fixture(scope="module")
def uneven():
    ws = [W.make_workload(n) for n in ("cube40", "ball60", "slab120")]
    return [(w, pat.Problem.from_workload(w)) for w in ws]


def test_uneven_fullsize_forward_sampled(uneven):
    """One forward sweep per mesh (16 float32 RHS): sampled RHS against the oracle, 1e-4 of the largest output."""
    for w, G in uneven:
        O = oracle.Problem.from_workload(w)
        p0 = np.random.default_rng(30).standard_normal((16, w.n_nodes))
        dev_in = _dev(p0, torch.float32)
        y = pat.pat_forward(G, dev_in).cpu().numpy().astype(np.float64)
        ref = O.forward(dev_in[3].cpu().numpy().astype(np.float64))
        err = float(np.abs(y[3] - ref).max() / np.abs(ref).max())
        print(f"{w.name} N={w.n_nodes}: forward f32 rhs 3 rel max err {err:.2e}", flush=True)
        assert err < 1e-4


def test_uneven_fullsize_batch_equals_single(uneven):
    probs = [G for _, G in uneven]
    B = pat.Batch(probs)
    rb, us = B.autotune(16, "f32")
    print(f"uneven batch autotuned rb={rb}, priced {us:.0f} us per merged step pair", flush=True)
    ys, sig = [], []
    for w, G in uneven:
        p0 = _dev(w.p0_true[None], torch.float64)
        Y = pat.pat_forward(G, p0)[0]
        ys.append(Y.contiguous())
        sig.append(float(0.01 * torch.linalg.norm(Y) / np.sqrt(Y.numel())))
    outs = pat.rto_sample_batch(B, ys, None, None, sig, 0.01, 3, sweep_prec="f32", n_samples=16, seed=7)
    for (w, G), y, s, o in zip(uneven, ys, sig, outs):
        ref = pat.rto_sample(G, y, None, None, s, 0.01, 3, sweep_prec="f32", rhs_block=rb, n_samples=16, seed=7)
        assert torch.equal(o["samples"], ref["samples"]), w.name
        assert torch.isfinite(o["std"]).all()
