"""The one-vector (three-level) form of the sweeps, which the GPU step kernels carry, against the
oracle's literal Stormer-Verlet substeps (Sec. 3 eq. (fully-discrete); Sec. 5.1 eq. (adjoint-verlet)
within the recursion (backward-recursion)).

CPU only: oracle/float32_floor.py's ThreeLevel, run in float64, must reproduce the oracle's forward
map G and its transpose to rounding.  This checks the elimination of the velocity (forward) and of
p_hat (transposed), the start values S^{-1} = S^0 = p^0 and q_{-1} = 0, q_0 = (dt/2m) Pi^T yhat^{N_T},
the sampled pressure p^{n+1} = (S^n + S^{n+1})/2 and the closing formula of the transposed sweep,
independently of the GPU code.  In float32 it stays within the rounding floor of a float32 sweep.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.float32_floor import ThreeLevel


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["cube8_tiny", "ball16", "box12"])
def test_three_level_equals_the_substeps(name):
    w = W.make_workload(name)
    O = oracle.Problem.from_workload(w)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, O.n_nodes))
    yh = rng.standard_normal((3, O.n_steps, O.n_obs))
    y64, a64 = O.forward(x), O.adjoint(yh)
    t64 = ThreeLevel(O, np.float64)
    assert _rel(t64.forward(x), y64) < 1e-13
    assert _rel(t64.adjoint(yh), a64) < 1e-13
    t32 = ThreeLevel(O, np.float32)
    assert _rel(t32.forward(x), y64) < 1e-5
    assert _rel(t32.adjoint(yh), a64) < 1e-5


@pytest.mark.parametrize("n_steps", [1, 2, 3])
def test_three_level_short_sweeps(n_steps):
    """The start values and the closing formula alone (one step: no recurrence step at all)."""
    w = W.make_workload("ball16")
    O = oracle.Problem.from_workload(w, n_steps=n_steps)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, O.n_nodes))
    yh = rng.standard_normal((2, n_steps, O.n_obs))
    t = ThreeLevel(O, np.float64)
    assert _rel(t.forward(x), O.forward(x)) < 1e-13
    assert _rel(t.adjoint(yh), O.adjoint(yh)) < 1e-13


def test_three_level_catches_a_wrong_start():
    """A plausible slip, starting the transposed recurrence with q_{-1} = q_0 (as the forward
    starts S^{-1} = S^0), leaves a visible error: the pin above is not vacuous."""
    w = W.make_workload("ball16")
    O = oracle.Problem.from_workload(w, n_steps=20)
    rng = np.random.default_rng(5)
    yh = rng.standard_normal((1, 20, O.n_obs))
    t = ThreeLevel(O, np.float64)
    good = t.adjoint(yh)
    step = t._step
    t._step = lambda S, Sp, src: step(S, S if Sp is not None and not Sp.any() else Sp, src)
    bad = t.adjoint(yh)
    assert _rel(good, O.adjoint(yh)) < 1e-13
    assert _rel(bad, O.adjoint(yh)) > 1e-3
