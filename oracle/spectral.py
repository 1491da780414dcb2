"""Oracle for the Whittle-Matern Fourier-spectral prior and latent-space RTO.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): plain, slow float64 numpy;
shares no code with the GPU library.

Prior (Sec. 4.1.2, eq. (matern-cov-op); set-up of Sec. 6.4).  On a periodic box
[lo, lo + side)^3 with n points per axis (spacing h = side/n) a latent white-noise
vector w ~ N(0, I) of length n^3 defines the grid field

    u = F^* diag(a) F w,   a(k) = c (ell^-2 + |k|^2)^(-expo/2),

F the unitary 3D DFT, k = 2 pi (integer frequency) / side.  Its covariance
F^* diag(a^2) F is the discrete counterpart of sigma^2 Z^-1 (ell^-2 I - Delta)^-expo
with expo = nu + d/2; c is set so that the pointwise variance (1/n^3) sum_k a(k)^2
equals sigma^2 (the normalisation the constant Z stands for).  The mesh field is
p0 = I_h u with I_h trilinear interpolation from the grid to the mesh nodes, so
p0 = P w with P = I_h F^* diag(a) F.

Latent RTO (Sec. 6.4: the optimisation runs in the latent space of the Fourier
representation): with the latent prior N(0, I) the extended problem of eq.
(extended-matrices) becomes G_ext = [G P / sigma ; I], b = [y/sigma + eta ; xi]
with xi of length n^3.  Each sample solves min ||G_ext w - b|| by CGLS with full
reorthogonalisation of the normal-equation residuals (as the FE-prior oracle),
and maps back p0 = P w.

Grid ordering: w[(k*n + j)*n + i] is the point (lo + i h, lo + j h, lo + k h).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class SpectralPrior:
    def __init__(self, n: int, lo: float, side: float, ell: float, sigma: float, expo: float = 3.0):
        self.n, self.lo, self.side, self.ell, self.sigma, self.expo = int(n), float(lo), float(side), float(ell), \
            float(sigma), float(expo)
        self.h = self.side / self.n
        self.size = self.n ** 3

    def amplitude(self) -> np.ndarray:
        """a(k) on the DFT grid, shape (n, n, n) with axes (z, y, x)."""
        k1 = 2.0 * np.pi * np.fft.fftfreq(self.n, d=self.h)
        kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
        base = (self.ell ** -2 + kx ** 2 + ky ** 2 + kz ** 2) ** (-self.expo / 2.0)
        c = self.sigma * np.sqrt(self.size / np.sum(base ** 2))
        return c * base

    def field(self, w: np.ndarray) -> np.ndarray:
        """u = F^* diag(a) F w on the grid for w [R][n^3] (or [n^3])."""
        single = np.ndim(w) == 1
        W = np.atleast_2d(w).reshape(-1, self.n, self.n, self.n)
        U = np.fft.ifftn(self.amplitude()[None] * np.fft.fftn(W, axes=(1, 2, 3)), axes=(1, 2, 3)).real
        U = U.reshape(-1, self.size)
        return U[0] if single else U

    def interp_matrix(self, coords: np.ndarray) -> sp.csr_matrix:
        """Trilinear interpolation I_h from the (periodic) grid to points [N][3]."""
        t = (np.asarray(coords, dtype=np.float64) - self.lo) / self.h
        if np.any(t < 0) or np.any(t >= self.n):
            raise ValueError("mesh nodes must lie inside the grid box")
        i0 = np.floor(t).astype(np.int64)
        f = t - i0
        rows, cols, vals = [], [], []
        N = t.shape[0]
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    wgt = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                           * (f[:, 2] if dz else 1 - f[:, 2]))
                    ix = (i0[:, 0] + dx) % self.n
                    iy = (i0[:, 1] + dy) % self.n
                    iz = (i0[:, 2] + dz) % self.n
                    rows.append(np.arange(N))
                    cols.append((iz * self.n + iy) * self.n + ix)
                    vals.append(wgt)
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, self.size))

    def apply(self, w: np.ndarray, I: sp.csr_matrix) -> np.ndarray:
        """p0 = P w = I_h u(w); w [R][n^3] -> [R][N]."""
        return np.asarray((I @ np.atleast_2d(self.field(w)).T).T)

    def apply_t(self, v: np.ndarray, I: sp.csr_matrix) -> np.ndarray:
        """P^T v = F^* diag(a) F I_h^T v; v [R][N] -> [R][n^3] (the filter is symmetric)."""
        g = np.asarray((I.T @ np.atleast_2d(v).T).T)
        return np.atleast_2d(self.field(g))


def latent_rto(problem, prior: SpectralPrior, I: sp.csr_matrix, yobs: np.ndarray, sigma: float, n_iter: int,
               eta: np.ndarray, xi: np.ndarray, reorth: bool = True, sweeps: str = "f64"):
    """Latent-space RTO samples: returns (p0 samples [S][N], latent samples [S][n^3], resid [S][n_iter+1]).

    eta [S][N_T][N_obs], xi [S][n^3].  CGLS on G_ext = [G P / sigma ; I] from w = 0.
    sweeps = "f32" runs the wave sweeps with float32 state and arithmetic (their inputs rounded
    to float32), everything else in float64: the rounding floor of a float32-sweep solver."""
    S = xi.shape[0]
    isig = 1.0 / sigma
    fwd, adj = (problem.forward, problem.adjoint) if sweeps == "f64" else (problem.forward_f32, problem.adjoint_f32)

    def gext(d):
        return isig * fwd(prior.apply(d, I)), d.copy()

    def gext_t(rd, rp):
        return isig * prior.apply_t(adj(rd), I) + rp

    def sq(a):
        return np.sum(a.reshape(a.shape[0], -1) ** 2, axis=1)

    x = np.zeros_like(xi)
    rd = yobs[None] * isig + eta
    rp = xi.copy()
    resid = np.empty((S, n_iter + 1))
    resid[:, 0] = np.sqrt(sq(rd) + sq(rp))
    s = gext_t(rd, rp)
    gamma = sq(s)
    Q = [s / np.sqrt(gamma)[:, None]] if reorth else []
    d = s.copy()
    for k in range(1, n_iter + 1):
        qd, qp = gext(d)
        delta = sq(qd) + sq(qp)
        alpha = np.where(delta > 0, gamma / np.where(delta > 0, delta, 1.0), 0.0)
        x += alpha[:, None] * d
        rd -= alpha[:, None, None] * qd
        rp -= alpha[:, None] * qp
        resid[:, k] = np.sqrt(sq(rd) + sq(rp))
        if k == n_iter:
            break
        s = gext_t(rd, rp)
        if reorth:
            for _ in range(2):
                coef = [np.sum(qj * s, axis=1) for qj in Q]
                for qj, cj in zip(Q, coef):
                    s -= cj[:, None] * qj
        gnew = sq(s)
        beta = np.where(gamma > 0, gnew / np.where(gamma > 0, gamma, 1.0), 0.0)
        if reorth:
            Q.append(s / np.sqrt(np.where(gnew > 0, gnew, 1.0))[:, None])
        d = s + beta[:, None] * d
        gamma = gnew
    return prior.apply(x, I), x, resid


def latent_residual(problem, prior: SpectralPrior, I: sp.csr_matrix, w: np.ndarray, yobs: np.ndarray, sigma: float,
                    eta: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """||G_ext w - b||_2 per latent sample w [S][n^3] (Sec. 5 eq. (lsqr-residual) with G_ext = [G P / sigma ; I],
    b = [y/sigma + eta ; xi]): data part from the float64 forward map of p0 = P w, prior part w - xi."""
    w = np.atleast_2d(w)
    rd = problem.forward(prior.apply(w, I)) / sigma - yobs[None] / sigma - np.reshape(eta, (w.shape[0],) + yobs.shape)
    rp = w - np.reshape(xi, w.shape)
    return np.sqrt(np.sum(rd.reshape(w.shape[0], -1) ** 2, axis=1) + np.sum(rp ** 2, axis=1))
