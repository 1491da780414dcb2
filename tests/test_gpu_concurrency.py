"""Distinct handles are independent: two problems sampled at once from two host
threads, each on its own stream (default priority), give bit for bit the results
of running them one after the other.  Both calls build their sweep graphs inside
the threads (first use of the handles), so graph capture runs concurrently too.
"""
import threading

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pat = pytest.importorskip("paper_2607_21373_amd.pat")


def _inputs(name):
    w = W.make_workload(name)
    O = oracle.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    return w, torch.as_tensor(yobs, device="cuda"), sigma


def _run(G, w, y, sigma, seed):
    return pat.rto_sample(G, y, None, None, sigma, w.prior_a, 10, sweep_prec="f32", rhs_block=16, n_samples=20,
                          seed=seed, resid=True)


def test_two_handles_two_threads_two_streams():
    cases = [_inputs("ball16"), _inputs("box12")]
    # reference: fresh handles, one call after the other on the default stream
    ref = []
    for k, (w, y, sigma) in enumerate(cases):
        G = pat.Problem.from_workload(w)
        ref.append(_run(G, w, y, sigma, k + 1))
    torch.cuda.synchronize()

    handles = [pat.Problem.from_workload(w) for w, _, _ in cases]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out, err = [None, None], [None, None]
    start = threading.Barrier(2)

    def work(k):
        try:
            w, y, sigma = cases[k]
            start.wait()
            with torch.cuda.stream(streams[k]):
                streams[k].wait_stream(torch.cuda.default_stream())
                out[k] = _run(handles[k], w, y, sigma, k + 1)
            streams[k].synchronize()
        except Exception as e:  # reported below, in the main thread
            err[k] = e

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=240)
    assert not any(t.is_alive() for t in threads), "a sampling thread did not finish"
    assert err == [None, None], err
    torch.cuda.synchronize()
    for k in range(2):
        for key in ("samples", "mean", "std", "resid"):
            assert torch.equal(out[k][key], ref[k][key]), (k, key)
        assert np.isfinite(out[k]["std"].cpu().numpy()).all()
