"""Plain CPU FP64 oracle for the 3D photoacoustic RTO sampler (arXiv 2607.21373).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and the
two share no code.  The arithmetic lives in ``pat_oracle.c`` (plain loops,
float64, no FMA contraction); this module only marshals NumPy arrays.

Layouts at this interface follow the GPU library's user-facing conventions:
  p0, p      [R][N]            one row per right-hand side
  y, yhat    [R][N_T][N_obs]   time-major data of each right-hand side
  eta        [S][N_T][N_obs],  xi [S][N]
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)
_fp = ctypes.POINTER(ctypes.c_float)


def build() -> str:
    """Compile the oracle with gcc (float64, -ffp-contract=off, OpenMP)."""
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.c_int, _dp, ctypes.c_int64, _ip, _dp, ctypes.c_int, ctypes.c_int,
                               _ip, _dp, ctypes.c_double, ctypes.c_int]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_nnz.restype = ctypes.c_int64
    lib.orc_nnz.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_get_csr.argtypes = [ctypes.c_void_p, ctypes.c_int, _lp, _ip, _dp]
    lib.orc_get_mass.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_get_sensors.argtypes = [ctypes.c_void_p, _ip, _dp]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_forward_f32.argtypes = [ctypes.c_void_p, ctypes.c_int, _fp, _fp]
    lib.orc_adjoint_f32.argtypes = [ctypes.c_void_p, ctypes.c_int, _fp, _fp]
    lib.orc_step_transpose.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_forward.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    lib.orc_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    lib.orc_prior_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp]
    lib.orc_prior_apply_transpose.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp]
    lib.orc_cgls.restype = ctypes.c_int
    lib.orc_cgls.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.orc_lsqr.restype = ctypes.c_int
    lib.orc_lsqr.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    lib.orc_rto.restype = ctypes.c_int
    lib.orc_rto.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
    lib.orc_stats.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
    _u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.orc_philox4x64.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_normals.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _dp]
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray], t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


class Problem:
    """Assembled discrete PAT problem (mesh, wave speed, boundary, sensors, dt, N_T)."""

    def __init__(self, coords, tets, c_tet=None, absorbing=True, dt=0.01, n_steps=100,
                 sensor_nodes=None, sensor_pos=None):
        lib = _load()
        self.coords = _f64(coords)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.c_tet = None if c_tet is None else _f64(c_tet)
        self.n_nodes = int(self.coords.shape[0])
        self.n_steps = int(n_steps)
        self.dt = float(dt)
        if (sensor_nodes is None) == (sensor_pos is None):
            raise ValueError("give exactly one of sensor_nodes and sensor_pos")
        sn = None if sensor_nodes is None else np.ascontiguousarray(sensor_nodes, dtype=np.int32)
        sp = None if sensor_pos is None else _f64(sensor_pos)
        self.n_obs = int(sn.size if sn is not None else sp.shape[0])
        h = lib.orc_create(self.n_nodes, _ptr(self.coords), int(self.tets.shape[0]), _ptr(self.tets, _ip),
                           _ptr(self.c_tet), int(bool(absorbing)), self.n_obs, _ptr(sn, _ip), _ptr(sp),
                           self.dt, self.n_steps)
        if not h:
            raise ValueError("oracle problem creation failed (sensor outside the mesh or bad ids)")
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_workload(cls, w, n_steps: Optional[int] = None):
        return cls(w.coords, w.tets, w.c_tet, w.absorbing, w.dt, w.n_steps if n_steps is None else n_steps,
                   sensor_nodes=w.sensor_nodes, sensor_pos=w.sensor_pos)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # -- assembled operators (for tests) ---------------------------------
    def csr(self, which: str):
        """Return (rowptr, col, val) of 'K', 'K1' or 'B'."""
        w = {"K": 0, "K1": 1, "B": 2}[which]
        lib = _load()
        nnz = int(lib.orc_nnz(self._h, w))
        rp = np.empty(self.n_nodes + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        val = np.empty(max(nnz, 1), dtype=np.float64)
        lib.orc_get_csr(self._h, w, _ptr(rp, _lp), _ptr(col, _ip), _ptr(val))
        return rp, col[:nnz], val[:nnz]

    def matrix(self, which: str):
        import scipy.sparse as sp
        rp, col, val = self.csr(which)
        return sp.csr_matrix((val, col, rp), shape=(self.n_nodes, self.n_nodes))

    def lumped_mass(self) -> np.ndarray:
        m = np.empty(self.n_nodes)
        _load().orc_get_mass(self._h, _ptr(m))
        return m

    def sensors(self):
        nodes = np.empty((self.n_obs, 4), dtype=np.int32)
        w = np.empty((self.n_obs, 4))
        _load().orc_get_sensors(self._h, _ptr(nodes, _ip), _ptr(w))
        return nodes, w

    # -- time stepping ----------------------------------------------------
    def step(self, p: np.ndarray, v: np.ndarray):
        """One forward step on [R][N] arrays; returns new (p, v)."""
        p = np.atleast_2d(p); v = np.atleast_2d(v)
        R = p.shape[0]
        pn, vn = np.array(p.T, dtype=np.float64, order="C"), np.array(v.T, dtype=np.float64, order="C")
        work = np.empty(2 * self.n_nodes * R)
        _load().orc_step(self._h, R, _ptr(pn), _ptr(vn), _ptr(work))
        return pn.T.copy(), vn.T.copy()

    def step_transpose(self, ph: np.ndarray, vh: np.ndarray):
        """One transpose step (A_dt^T) on [R][N] arrays; returns new (ph, vh)."""
        ph = np.atleast_2d(ph); vh = np.atleast_2d(vh)
        R = ph.shape[0]
        a, b = np.array(ph.T, dtype=np.float64, order="C"), np.array(vh.T, dtype=np.float64, order="C")
        work = np.empty(self.n_nodes * R)
        _load().orc_step_transpose(self._h, R, _ptr(a), _ptr(b), _ptr(work))
        return a.T.copy(), b.T.copy()

    def forward(self, p0: np.ndarray) -> np.ndarray:
        """y = G p0 for p0 [R][N] (or [N]); returns [R][N_T][N_obs] (or [N_T][N_obs])."""
        single = np.ndim(p0) == 1
        p0 = np.atleast_2d(p0)
        R = p0.shape[0]
        x = _f64(p0.T)
        y = np.empty((self.n_steps, self.n_obs, R))
        _load().orc_forward(self._h, R, _ptr(x), _ptr(y))
        out = np.moveaxis(y, 2, 0)
        return np.ascontiguousarray(out[0] if single else out)

    def forward_f32(self, p0: np.ndarray) -> np.ndarray:
        """forward() with float32 state and arithmetic (rounding-floor studies only); returns float64."""
        p0 = np.atleast_2d(p0)
        R = p0.shape[0]
        x = np.ascontiguousarray(p0.T, dtype=np.float32)
        y = np.empty((self.n_steps, self.n_obs, R), dtype=np.float32)
        _load().orc_forward_f32(self._h, R, x.ctypes.data_as(_fp), y.ctypes.data_as(_fp))
        return np.ascontiguousarray(np.moveaxis(y, 2, 0)).astype(np.float64)

    def adjoint_f32(self, yhat: np.ndarray) -> np.ndarray:
        """adjoint() with float32 state and arithmetic (rounding-floor studies only); returns float64."""
        yh = yhat[None] if np.ndim(yhat) == 2 else yhat
        R = yh.shape[0]
        a = np.ascontiguousarray(np.moveaxis(yh, 0, 2), dtype=np.float32)
        p = np.empty((self.n_nodes, R), dtype=np.float32)
        _load().orc_adjoint_f32(self._h, R, a.ctypes.data_as(_fp), p.ctypes.data_as(_fp))
        return np.ascontiguousarray(p.T).astype(np.float64)

    def adjoint(self, yhat: np.ndarray) -> np.ndarray:
        """p = G^T yhat for yhat [R][N_T][N_obs] (or [N_T][N_obs]); returns [R][N] (or [N])."""
        single = np.ndim(yhat) == 2
        yh = yhat[None] if single else yhat
        R = yh.shape[0]
        a = _f64(np.moveaxis(yh, 0, 2))
        p = np.empty((self.n_nodes, R))
        _load().orc_adjoint(self._h, R, _ptr(a), _ptr(p))
        out = p.T
        return np.ascontiguousarray(out[0] if single else out)

    def prior_apply(self, x: np.ndarray, a: float, transpose: bool = False) -> np.ndarray:
        """L x (or L^T x) for L = M_L^{-1/2}(M_L + a K1); x [R][N] or [N]."""
        single = np.ndim(x) == 1
        x2 = np.atleast_2d(x)
        R = x2.shape[0]
        xi = _f64(x2.T)
        y = np.empty_like(xi)
        f = _load().orc_prior_apply_transpose if transpose else _load().orc_prior_apply
        f(self._h, R, float(a), _ptr(xi), _ptr(y))
        return np.ascontiguousarray(y.T[0] if single else y.T)

    def extended_residual(self, p: np.ndarray, yobs: np.ndarray, sigma: float, prior_a: float, eta: np.ndarray,
                          xi: np.ndarray) -> np.ndarray:
        """||G_ext p - b||_2 per sample (Sec. 5 eq. (lsqr-residual)), b = (yobs/sigma + eta, xi):
        data part (G p - yobs - sigma eta)/sigma from the float64 forward map, prior part
        L p - xi (L p_prior = xi).  p [S][N], eta [S][N_T][N_obs], xi [S][N]; returns [S]."""
        p = np.atleast_2d(p)
        rd = (self.forward(p) - yobs[None] - sigma * np.reshape(eta, (p.shape[0],) + yobs.shape)) / sigma
        rp = self.prior_apply(p, prior_a) - np.reshape(xi, p.shape)
        return np.sqrt(np.sum(rd.reshape(p.shape[0], -1) ** 2, axis=1) + np.sum(rp ** 2, axis=1))

    # -- least squares and sampling ----------------------------------------
    def cgls(self, bd: np.ndarray, bp: np.ndarray, sigma: float, prior_a: float, n_iter: int,
             reorth: bool = True, solver: str = "cgls", diag: bool = False):
        """Least squares min ||G_ext x - b||, b = (bd [R][N_T][N_obs], bp [R][N]), by CGLS or LSQR.

        Returns (x [R][N], resid [R][n_iter+1]) and, with diag=True, also
        [R][n_iter+1][2] = (||r_d||, ||r_p||) per iteration."""
        R = bp.shape[0]
        bdi = _f64(np.moveaxis(bd, 0, 2))
        bpi = _f64(bp.T)
        x = np.empty((self.n_nodes, R))
        res = np.empty((R, n_iter + 1))
        dg = np.empty((R, n_iter + 1, 2))
        f = {"cgls": _load().orc_cgls, "lsqr": _load().orc_lsqr}[solver]
        rc = f(self._h, R, float(sigma), float(prior_a), int(n_iter), int(bool(reorth)),
               _ptr(bdi), _ptr(bpi), _ptr(x), _ptr(res), _ptr(dg))
        if rc != 0:
            raise MemoryError("oracle least-squares solve could not allocate its workspace")
        out = (np.ascontiguousarray(x.T), res)
        return out + (dg,) if diag else out

    def lsqr(self, bd, bp, sigma, prior_a, n_iter, reorth=True, diag=False):
        return self.cgls(bd, bp, sigma, prior_a, n_iter, reorth, solver="lsqr", diag=diag)

    def rto(self, yobs: np.ndarray, sigma: float, prior_a: float, n_iter: int, eta: np.ndarray, xi: np.ndarray,
            reorth: bool = True, solver: str = "cgls", diag: bool = False):
        """RTO samples (Algorithm 1): returns (samples [S][N], resid [S][n_iter+1]) [, diag]."""
        S = xi.shape[0]
        ya = _f64(yobs)
        ea = _f64(np.moveaxis(eta, 0, 2))
        xa = _f64(xi.T)
        out = np.empty((self.n_nodes, S))
        res = np.empty((S, n_iter + 1))
        dg = np.empty((S, n_iter + 1, 2))
        rc = _load().orc_rto(self._h, S, _ptr(ya), float(sigma), float(prior_a), int(n_iter), int(bool(reorth)),
                             _ptr(ea), _ptr(xa), _ptr(out), _ptr(res), {"cgls": 0, "lsqr": 1}[solver], _ptr(dg))
        if rc != 0:
            raise MemoryError("oracle RTO could not allocate its workspace")
        ret = (np.ascontiguousarray(out.T), res)
        return ret + (dg,) if diag else ret


def stats(samples: np.ndarray):
    """Pointwise mean and std (1/(S-1)) of samples [S][N], eq. (ergodic)."""
    S, N = samples.shape
    a = _f64(samples.T)
    mean = np.empty(N); std = np.empty(N)
    _load().orc_stats(N, S, _ptr(a), _ptr(mean), _ptr(std))
    return mean, std


def philox4x64(ctr, key) -> np.ndarray:
    """Philox4x64-10 block (Salmon et al., SC'11) of counter ctr[4] under key[2]."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, dtype=np.uint64)
    u = ctypes.POINTER(ctypes.c_uint64)
    _load().orc_philox4x64(c.ctypes.data_as(u), k.ctypes.data_as(u), out.ctypes.data_as(u))
    return out


def normals(seed: int, kind: int, k0: int, S: int, length: int) -> np.ndarray:
    """[S][length] standard normals of streams (seed, kind, k0..k0+S-1): Philox4x64-10 + Box-Muller."""
    out = np.empty((S, length))
    _load().orc_normals(int(seed), int(kind), int(k0), int(S), int(length), _ptr(out))
    return out


def rto_normals(seed: int, S: int, n_steps: int, n_obs: int, n_nodes: int):
    """eta [S][N_T][N_obs] (kind 0) and xi [S][N] (kind 1) as the sampler draws them itself."""
    return (normals(seed, 0, 0, S, n_steps * n_obs).reshape(S, n_steps, n_obs), normals(seed, 1, 0, S, n_nodes))


def noise_sigma(Y: np.ndarray, eta0: np.ndarray, d_noise: float, rule: str) -> float:
    """Absolute noise level of the synthetic data.

    rule "l2": sigma = d_noise * ||Y|| / ||eta0|| (Sec. 2, eq. (noise-model); the
    dt weights of the discrete L2(0,T; l2) norms cancel in the ratio).
    rule "max": sigma = d_noise * max|Y|.
    """
    if rule == "l2":
        return float(d_noise * np.sqrt(np.sum(Y * Y)) / np.sqrt(np.sum(eta0 * eta0)))
    if rule == "max":
        return float(d_noise * np.max(np.abs(Y)))
    raise ValueError(rule)


def synthesize(problem: Problem, w, eta0: Optional[np.ndarray] = None):
    """Noise-free data Y = G p0_true, sigma, and y_obs = Y + sigma * eta0."""
    import workloads
    Y = problem.forward(w.p0_true)
    if eta0 is None:
        eta0 = workloads.noise_draw(problem.n_steps, problem.n_obs, w.noise_seed)
    sigma = noise_sigma(Y, eta0, w.d_noise, w.noise_rule)
    return Y, Y + sigma * eta0, sigma


def diagnostics(diag: np.ndarray, n_data: int, tau: float = 1.0) -> dict:
    """Convergence diagnostics of Sec. 6.1 from a history diag [S][n_iter+1][2] of
    (||r_d||, ||r_p||), r_d the whitened data residual: per iteration the normalised data
    misfit ||r_d|| / sqrt(N_T N_obs) (1 at the discrepancy level), the prior part
    ||r_p|| / ||b|| and the extended residual ||r|| / ||b|| (||b|| = the residual at x = 0),
    and the first iteration meeting the discrepancy principle ||r_d|| <= tau sqrt(N_T N_obs)
    (-1 if none)."""
    d = np.asarray(diag, dtype=np.float64)
    if d.ndim != 3 or d.shape[2] != 2:
        raise ValueError("diag must have shape [S][n_iter+1][2]")
    S, n1 = d.shape[0], d.shape[1]
    out = {"data": np.empty((S, n1)), "prior": np.empty((S, n1)), "extended": np.empty((S, n1)),
           "discrepancy": np.full(S, -1, dtype=np.int32)}
    level = tau * math.sqrt(n_data)
    for k in range(S):
        b = math.sqrt(d[k, 0, 0] ** 2 + d[k, 0, 1] ** 2)
        ib = 1.0 / b if b > 0 else 1.0
        for j in range(n1):
            nd, npr = d[k, j, 0], d[k, j, 1]
            out["data"][k, j] = nd / math.sqrt(n_data)
            out["prior"][k, j] = npr * ib
            out["extended"][k, j] = math.sqrt(nd * nd + npr * npr) * ib
            if out["discrepancy"][k] < 0 and nd <= level:
                out["discrepancy"][k] = j
    return out
