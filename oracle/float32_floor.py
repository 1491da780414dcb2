"""Float32 rounding floor of the staggered Stormer-Verlet sweeps.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): numpy float32 arithmetic,
shares no code with the GPU library.

The GPU sweeps carry the staggered state (p^{n+1/2}, v^n) of Sec. 3 eq.
(fully-discrete) with lumped mass, and for the transpose (p_hat, M_L^{-1}(v_hat +
dt/2 p_hat)) of Sec. 5.1 eq. (adjoint-verlet).  This module runs the same two
recurrences with every stored value in float32 (matrices, dt/m, state, data), so
that the rounding floor of a float32 path can be measured on the CPU where a
float32 result is poorly conditioned.  It is never used to produce an expected
value: the references stay the float64 oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class StaggeredFloat32:
    """forward(p0) / adjoint(yhat) with float32 staggered steps; inputs and outputs float64."""

    def __init__(self, problem):
        self.n_nodes, self.n_steps, self.n_obs = problem.n_nodes, problem.n_steps, problem.n_obs
        self.K = problem.matrix("K").astype(np.float32).tocsr()
        self.B = problem.matrix("B").astype(np.float32).tocsr()
        self.dm = (problem.dt / problem.lumped_mass()).astype(np.float32)[:, None]
        self.dt = np.float32(problem.dt)
        self.hdt = np.float32(0.5 * problem.dt)
        nodes, w = problem.sensors()
        Pi = sp.csr_matrix((w.ravel(), (np.repeat(np.arange(self.n_obs), 4), nodes.ravel())),
                           shape=(self.n_obs, self.n_nodes))
        self.Pi = Pi.astype(np.float32).tocsr()
        self.PiT = Pi.T.tocsr().astype(np.float32)

    def forward(self, p0):
        p0 = np.atleast_2d(p0)
        P = np.ascontiguousarray(p0.T, dtype=np.float32)   # p^{1/2} = p^0 (v^0 = 0)
        V = np.zeros_like(P)
        Y = np.empty((self.n_steps, self.n_obs, P.shape[1]), np.float32)
        for n in range(self.n_steps):
            V = V - self.dm * (self.K @ P + self.B @ V)    # v^{n+1}
            P = P + self.dt * V                            # p^{n+3/2}
            Y[n] = self.Pi @ (P - self.hdt * V)            # Pi p^{n+1}
        return np.moveaxis(Y, 2, 0).astype(np.float64)

    def adjoint(self, yhat):
        Y = np.moveaxis(np.asarray(yhat), 0, 2).astype(np.float32)   # [N_T][N_obs][R]
        NT = self.n_steps
        PH = self.PiT @ Y[NT - 1]
        Q = np.float32(0.5) * self.dm * PH
        for n in range(NT, 0, -1):
            PH = PH - self.dt * (self.K @ Q)
            if n > 1:
                inj = self.PiT @ Y[n - 2]
                Q = Q - self.dm * (self.B @ Q) + self.dm * (PH + np.float32(0.5) * inj)
                PH = PH + inj
        return PH.T.astype(np.float64)
