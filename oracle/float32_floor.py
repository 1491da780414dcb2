"""Rounding floors of the reduced-precision Stormer-Verlet sweeps.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): numpy arithmetic, shares no
code with the GPU library.

Two ways of carrying the lumped-mass recurrences of Sec. 3 eq. (fully-discrete)
and Sec. 5.1 eq. (adjoint-verlet), each run with every stored value in the chosen
type (matrices, dt/m, state, data), so that the rounding floor of a float32 path
can be measured on the CPU where a float32 result is poorly conditioned:

* StaggeredFloat32: the velocity form, state (p^{n+1/2}, v^n) forward and
  (p_hat, M_L^{-1}(v_hat + dt/2 p_hat)) transposed.
* ThreeLevel: one state vector per direction.  Forward, S^n = p^{n+1/2} with
  dt v^n = S^n - S^{n-1}; transposed, q = M_L^{-1}(v_hat + dt/2 p_hat) with p_hat
  recovered from two consecutive q.  In float64 it reproduces the oracle's maps
  to rounding, which checks the reformulation itself.

Neither is ever used to produce an expected value: the references stay the
float64 oracle.
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


class ThreeLevel:
    """forward(p0) / adjoint(yhat) in the one-vector (three-level) form, in `dtype`.

    Forward: eliminating v from the three substeps (p^{n+1/2} = p^n + dt/2 v^n, the
    velocity update, p^{n+1} = p^{n+1/2} + dt/2 v^{n+1}) with S^n = p^{n+1/2} gives
    dt v^n = S^n - S^{n-1} and
        S^{n+1} = S^n + (S^n - S^{n-1}) - (dt/m)(dt K S^n + B (S^n - S^{n-1})),
    with S^{-1} = S^0 = p^0 (v^0 = 0); the observed pressure is
    p^{n+1} = (S^n + S^{n+1})/2.
    Transposed: in the staggered transpose state (p_hat, q), each step back is
    p_hat -= dt K q, q += (dt/m)(p_hat - B q + inj/2), p_hat += inj.  Solving the
    q update for p_hat and substituting gives, with inj_j = Pi^T yhat^{N_T - j},
        q_{k+1} = q_k + (q_k - q_{k-1}) - (dt/m)(dt K q_k + B (q_k - q_{k-1}) - (inj_k + inj_{k+1})/2)
    from q_{-1} = 0, q_0 = (dt/2m) inj_0, and the result
        G^T yhat = (q_K - q_{K-1}) m/dt - (dt K q_K - B q_{K-1} - inj_K/2),  K = N_T - 1.
    """

    def __init__(self, problem, dtype=np.float32):
        self.t = np.dtype(dtype).type
        self.n_nodes, self.n_steps, self.n_obs = problem.n_nodes, problem.n_steps, problem.n_obs
        self.K = problem.matrix("K").astype(dtype).tocsr()
        self.B = problem.matrix("B").astype(dtype).tocsr()
        self.dm = (problem.dt / problem.lumped_mass()).astype(dtype)[:, None]
        self.dt = self.t(problem.dt)
        nodes, w = problem.sensors()
        Pi = sp.csr_matrix((w.ravel(), (np.repeat(np.arange(self.n_obs), 4), nodes.ravel())),
                           shape=(self.n_obs, self.n_nodes))
        self.Pi = Pi.astype(dtype).tocsr()
        self.PiT = Pi.T.tocsr().astype(dtype)

    def _step(self, S, Sp, src):
        d = S - Sp
        f = self.dt * (self.K @ S) + self.B @ d - src
        return S + (d - self.dm * f)

    def forward(self, p0):
        S = np.ascontiguousarray(np.atleast_2d(p0).T, dtype=self.t)
        Sp = S
        zero = self.t(0)
        Y = np.empty((self.n_steps, self.n_obs, S.shape[1]), self.t)
        for n in range(self.n_steps):
            Sn = self._step(S, Sp, zero)
            Y[n] = self.Pi @ (self.t(0.5) * (S + Sn))
            Sp, S = S, Sn
        return np.moveaxis(Y, 2, 0).astype(np.float64)

    def adjoint(self, yhat):
        Y = np.moveaxis(np.asarray(yhat), 0, 2).astype(self.t)   # [N_T][N_obs][R]
        NT = self.n_steps
        inj = lambda j: self.PiT @ Y[NT - 1 - j]                 # inj_j = Pi^T yhat^{N_T - j}
        half = self.t(0.5)
        q = half * self.dm * inj(0)
        qp = np.zeros_like(q)
        for k in range(NT - 1):
            q, qp = self._step(q, qp, half * (inj(k) + inj(k + 1))), q
        f = self.dt * (self.K @ q) - self.B @ qp - half * inj(NT - 1)
        return ((q - qp) / self.dm - f).T.astype(np.float64)
