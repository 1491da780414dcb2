"""Thin Python binding of libpat (``include/pat.h``).

Argument marshalling only: every step of the forward map, its transpose, the
CGLS solve and the statistics runs in libpat's HIP kernels.  Tensors are
PyTorch CUDA (HIP) tensors; work is enqueued on ``torch.cuda.current_stream()``.
There is no CPU fallback: importing this module without a built ``libpat.so``
raises, and every call needs a GPU.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
# Imported before libpat makes its first HIP call: a process whose first HIP user is
# libpat (a problem created before anything imported torch) later fails to
# initialise torch's GPU context ("No HIP GPUs are available").
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAT_LIB selects an alternative build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PAT_LIB") or os.path.join(_HERE, "libpat.so")

PAT_F64, PAT_F32 = 0, 1
_STATUS = {0: "PAT_OK", -1: "PAT_ERR_INVALID_ARG", -2: "PAT_ERR_UNSTABLE_DT", -3: "PAT_ERR_NONFINITE",
           -4: "PAT_ERR_OUT_OF_MEMORY", -5: "PAT_ERR_HIP", -6: "PAT_ERR_INTERNAL"}


class PatError(RuntimeError):
    """A libpat call returned a non-zero pat_status."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = _STATUS.get(code, str(code))


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int32), ("coords", ctypes.POINTER(ctypes.c_double)),
        ("n_tets", ctypes.c_int64), ("tets", ctypes.POINTER(ctypes.c_int32)),
        ("c_tet", ctypes.POINTER(ctypes.c_double)), ("absorbing", ctypes.c_int32),
        ("n_obs", ctypes.c_int32), ("sensor_nodes", ctypes.POINTER(ctypes.c_int32)),
        ("sensor_pos", ctypes.POINTER(ctypes.c_double)), ("dt", ctypes.c_double),
        ("n_steps", ctypes.c_int32), ("device", ctypes.c_int32), ("check_dt", ctypes.c_int32),
    ]


class ProblemInfo(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int32), ("n_obs", ctypes.c_int32), ("n_steps", ctypes.c_int32),
        ("n_tets", ctypes.c_int64), ("nnz_k", ctypes.c_int64), ("nnz_b", ctypes.c_int64),
        ("n_boundary_nodes", ctypes.c_int32), ("max_row_nnz", ctypes.c_int32),
        ("dt", ctypes.c_double), ("lambda_max", ctypes.c_double), ("device_bytes", ctypes.c_int64),
        ("b_stored", ctypes.c_int64),
    ]


class Profile(ctypes.Structure):
    _fields_ = [("fwd_ms", ctypes.c_double), ("adj_ms", ctypes.c_double), ("fwd_sweeps", ctypes.c_int64),
                ("adj_sweeps", ctypes.c_int64)]


class RtoParams(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double), ("prior_a", ctypes.c_double), ("n_iter", ctypes.c_int32),
        ("reorth", ctypes.c_int32), ("sweep_prec", ctypes.c_int), ("rhs_block", ctypes.c_int32),
        ("eta", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("solver", ctypes.c_int32), ("diag_hist", ctypes.c_void_p),
        ("seed", ctypes.c_uint64), ("sample0", ctypes.c_int64), ("prior", ctypes.c_int32),
        ("latent", ctypes.c_void_p), ("final_resid", ctypes.c_void_p),
    ]


PAT_CGLS, PAT_LSQR = 0, 1
PAT_PRIOR_FE, PAT_PRIOR_SPECTRAL = 0, 1


class SpectralDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("lo", ctypes.c_double * 3), ("side", ctypes.c_double),
                ("ell", ctypes.c_double), ("sigma", ctypes.c_double), ("expo", ctypes.c_double)]


# names exported by libpat (the C ABI in include/pat.h)
EXPORTS = ("pat_problem_create", "pat_problem_destroy", "pat_problem_get_info", "pat_forward", "pat_forward_noalloc",
           "pat_adjoint",
           "rto_sample", "pat_prior_apply", "pat_draw_normals", "pat_spectral_prior_set", "pat_spectral_apply",
           "pat_autotune", "pat_batch_create", "pat_batch_destroy", "pat_batch_autotune", "pat_batch_merge",
           "rto_sample_batch", "pat_solver_diagnostics", "pat_host_assemble", "pat_profile_enable",
           "pat_profile_get", "pat_sync",
           "pat_last_error", "pat_version")

_lib = None


def load() -> ctypes.CDLL:
    """Load libpat.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpat.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2607_21373_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.pat_problem_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(vp)]
    lib.pat_problem_destroy.argtypes = [vp]
    lib.pat_problem_get_info.argtypes = [vp, ctypes.POINTER(ProblemInfo)]
    lib.pat_forward.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_int, vp]
    lib.pat_forward_noalloc.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_int, vp]
    lib.pat_adjoint.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_int, vp]
    lib.rto_sample.argtypes = [vp, vp, ctypes.POINTER(RtoParams), ctypes.c_int64, vp, vp, vp, vp, vp]
    lib.pat_sync.argtypes = [vp]
    lib.pat_host_assemble.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(ctypes.c_int64)] + [vp] * 9
    lib.pat_profile_enable.argtypes = [vp, ctypes.c_int]
    lib.pat_prior_apply.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, vp, vp, vp]
    lib.pat_draw_normals.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     vp, vp]
    lib.pat_profile_get.argtypes = [vp, ctypes.POINTER(Profile)]
    i32p, f64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.pat_autotune.argtypes = [vp, ctypes.c_int64, ctypes.c_int, i32p, f64p, vp]
    lib.pat_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.pat_batch_destroy.argtypes = [vp]
    lib.pat_batch_merge.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.pat_spectral_prior_set.argtypes = [vp, ctypes.POINTER(SpectralDesc)]
    lib.pat_spectral_apply.argtypes = [vp, ctypes.c_int64, ctypes.c_int, vp, vp, vp]
    lib.pat_batch_autotune.argtypes = [vp, ctypes.c_int64, ctypes.c_int, i32p, f64p, vp]
    lib.rto_sample_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(RtoParams), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.pat_solver_diagnostics.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                           vp, vp, vp, vp, vp]
    lib.pat_last_error.restype = ctypes.c_char_p
    lib.pat_version.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f not in ("pat_last_error", "pat_version"):
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise PatError(rc, load().pat_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _prec(dtype):
    import torch
    if dtype == torch.float64:
        return PAT_F64
    if dtype == torch.float32:
        return PAT_F32
    raise TypeError("only float32 and float64 are supported")


def pat_problem_create(coords, tets, c_tet=None, absorbing=True, dt=0.01, n_steps=100, sensor_nodes=None,
                       sensor_pos=None, device: int = -1, check_dt: bool = True) -> "Problem":
    return Problem(coords, tets, c_tet, absorbing, dt, n_steps, sensor_nodes, sensor_pos, device, check_dt)


def _desc(coords, tets, c_tet, absorbing, dt, n_steps, sensor_nodes, sensor_pos, device, check_dt):
    """Fill a pat_problem_desc; returns (desc, arrays that must stay alive)."""
    keep = []

    def arr(a, dt_):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt_)
        keep.append(a)
        return a

    co, te = arr(coords, np.float64), arr(tets, np.int32)
    c = arr(c_tet, np.float64)
    sn, sp = arr(sensor_nodes, np.int32), arr(sensor_pos, np.float64)
    d = ProblemDesc()
    d.n_nodes = co.shape[0]
    d.coords = co.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_tets = te.shape[0]
    d.tets = te.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.c_tet = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if c is not None else None
    d.absorbing = int(bool(absorbing))
    d.n_obs = (sn.size if sn is not None else (sp.shape[0] if sp is not None else 0))
    d.sensor_nodes = sn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if sn is not None else None
    d.sensor_pos = sp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if sp is not None else None
    d.dt = float(dt)
    d.n_steps = int(n_steps)
    d.device = int(device)
    d.check_dt = int(bool(check_dt))
    return d, keep


def pat_host_assemble(coords, tets, c_tet=None, absorbing=True, dt=0.01, n_steps=100, sensor_nodes=None,
                      sensor_pos=None, check_dt: bool = True) -> dict:
    """Host-side assembly of libpat (no GPU needed): K, K1, B, M_L and sensor rows."""
    lib = load()
    d, keep = _desc(coords, tets, c_tet, absorbing, dt, n_steps, sensor_nodes, sensor_pos, -1, check_dt)
    nnz = ctypes.c_int64()
    _check(lib.pat_host_assemble(ctypes.byref(d), ctypes.byref(nnz), *([None] * 9)))
    N, O, Z = d.n_nodes, d.n_obs, nnz.value
    out = {"rowptr": np.empty(N + 1, np.int32), "col": np.empty(Z, np.int32), "K": np.empty(Z),
           "K1": np.empty(Z), "B": np.empty(Z), "mass": np.empty(N), "snode": np.empty((O, 4), np.int32),
           "sw": np.empty((O, 4)), "lambda_max": np.empty(1)}
    ptrs = [ctypes.c_void_p(out[k].ctypes.data) for k in
            ("rowptr", "col", "K", "K1", "B", "mass", "snode", "sw", "lambda_max")]
    _check(lib.pat_host_assemble(ctypes.byref(d), ctypes.byref(nnz), *ptrs))
    del keep
    out["lambda_max"] = float(out["lambda_max"][0])
    return out


class Problem:
    """Handle on a libpat problem (pat_problem_create / pat_problem_destroy)."""

    def __init__(self, coords, tets, c_tet=None, absorbing=True, dt=0.01, n_steps=100, sensor_nodes=None,
                 sensor_pos=None, device: int = -1, check_dt: bool = True):
        lib = load()
        d, keep = _desc(coords, tets, c_tet, absorbing, dt, n_steps, sensor_nodes, sensor_pos, device, check_dt)
        h = ctypes.c_void_p()
        self._h = None
        _check(lib.pat_problem_create(ctypes.byref(d), ctypes.byref(h)))
        del keep
        self._h = h
        info = self.info()
        self.n_nodes, self.n_obs, self.n_steps = info["n_nodes"], info["n_obs"], info["n_steps"]
        self.dt = info["dt"]

    @classmethod
    def from_workload(cls, w, n_steps: Optional[int] = None, device: int = -1, check_dt: bool = True):
        return cls(w.coords, w.tets, w.c_tet, w.absorbing, w.dt, w.n_steps if n_steps is None else n_steps,
                   sensor_nodes=w.sensor_nodes, sensor_pos=w.sensor_pos, device=device, check_dt=check_dt)

    def info(self) -> dict:
        out = ProblemInfo()
        _check(load().pat_problem_get_info(self._h, ctypes.byref(out)))
        return {name: getattr(out, name) for name, _ in ProblemInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().pat_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(load().pat_sync(self._h))

    def profile_enable(self, on: bool = True):
        _check(load().pat_profile_enable(self._h, int(bool(on))))

    def profile(self) -> dict:
        out = Profile()
        _check(load().pat_profile_get(self._h, ctypes.byref(out)))
        return {name: getattr(out, name) for name, _ in Profile._fields_}


def pat_forward(problem: Problem, p0, y=None):
    """Y = G p0 for p0 [R][N] (float32 or float64 CUDA tensor); returns y [R][N_T][N_obs]."""
    import torch
    R = p0.shape[0]
    if y is None:
        y = torch.empty((R, problem.n_steps, problem.n_obs), dtype=p0.dtype, device=p0.device)
    pp = _dev_ptr(p0, p0.dtype, (R, problem.n_nodes), "p0")
    yp = _dev_ptr(y, p0.dtype, (R, problem.n_steps, problem.n_obs), "y")
    _check(load().pat_forward(problem._h, R, pp, yp, _prec(p0.dtype), _stream()))
    return y


def pat_forward_noalloc(problem: Problem, p0, y):
    """pat_forward_noalloc: Y = G p0 into the caller's y [R][N_T][N_obs] with the library's
    fixed device scratch (no device allocation by the library)."""
    R = p0.shape[0]
    pp = _dev_ptr(p0, p0.dtype, (R, problem.n_nodes), "p0")
    yp = _dev_ptr(y, p0.dtype, (R, problem.n_steps, problem.n_obs), "y")
    _check(load().pat_forward_noalloc(problem._h, R, pp, yp, _prec(p0.dtype), _stream()))
    return y


def pat_adjoint(problem: Problem, yhat, p=None):
    """p = G^T yhat for yhat [R][N_T][N_obs]; returns p [R][N]."""
    import torch
    R = yhat.shape[0]
    if p is None:
        p = torch.empty((R, problem.n_nodes), dtype=yhat.dtype, device=yhat.device)
    yp = _dev_ptr(yhat, yhat.dtype, (R, problem.n_steps, problem.n_obs), "yhat")
    pp = _dev_ptr(p, yhat.dtype, (R, problem.n_nodes), "p")
    _check(load().pat_adjoint(problem._h, R, yp, pp, _prec(yhat.dtype), _stream()))
    return p


def pat_prior_apply(problem: Problem, x, prior_a: float, transpose: bool = False, y=None):
    """L x (or L^T x) for L = M_L^{-1/2}(M_L + a K1); x [R][N] float64 CUDA tensor."""
    import torch
    R = x.shape[0]
    if y is None:
        y = torch.empty_like(x)
    xp = _dev_ptr(x, torch.float64, (R, problem.n_nodes), "x")
    yp = _dev_ptr(y, torch.float64, (R, problem.n_nodes), "y")
    _check(load().pat_prior_apply(problem._h, R, float(prior_a), int(bool(transpose)), xp, yp, _stream()))
    return y


def spectral_prior_set(problem: Problem, n: int, lo, side: float, ell: float, sigma: float, expo: float = 3.0):
    """pat_spectral_prior_set: Whittle-Matern prior on an n^3 grid over [lo, lo + side)^3 (None clears)."""
    if n is None:
        _check(load().pat_spectral_prior_set(problem._h, None))
        problem.spectral_size = None
        return
    d = SpectralDesc()
    d.n = int(n)
    d.lo[0], d.lo[1], d.lo[2] = (float(v) for v in (lo if hasattr(lo, "__len__") else (lo, lo, lo)))
    d.side, d.ell, d.sigma, d.expo = float(side), float(ell), float(sigma), float(expo)
    _check(load().pat_spectral_prior_set(problem._h, ctypes.byref(d)))
    problem.spectral_size = int(n) ** 3


def spectral_apply(problem: Problem, x, transpose: bool = False):
    """y = P x (x [R][n^3] -> [R][N]) or P^T x (x [R][N] -> [R][n^3]), float64 CUDA tensors."""
    import torch
    G = getattr(problem, "spectral_size", None)
    if G is None:
        raise ValueError("no spectral prior set on this problem")
    R = x.shape[0]
    rows_in, rows_out = (problem.n_nodes, G) if transpose else (G, problem.n_nodes)
    xp = _dev_ptr(x, torch.float64, (R, rows_in), "x")
    y = torch.empty((R, rows_out), dtype=torch.float64, device=x.device)
    _check(load().pat_spectral_apply(problem._h, R, int(bool(transpose)), xp, ctypes.c_void_p(y.data_ptr()),
                                     _stream()))
    return y


def _rto_call(problem, y_obs, eta, xi, sigma, prior_a, n_iter, reorth, sweep_prec, rhs_block, stats, resid, samples,
              solver, diag, n_samples, seed, sample0, prior="fe", latent=False, final=False):
    """Allocate outputs and fill RtoParams for one problem; returns (prm, S, outputs, pointers)."""
    import torch
    f64 = torch.float64
    if (eta is None) != (xi is None):
        raise ValueError("pass both eta and xi, or neither")
    if xi is not None:
        S = xi.shape[0]
        dev = xi.device
    else:
        if n_samples is None:
            raise ValueError("n_samples is required when the library draws eta and xi")
        S = int(n_samples)
        dev = y_obs.device
    N, T, O = problem.n_nodes, problem.n_steps, problem.n_obs
    NX = N
    if prior == "spectral":
        NX = getattr(problem, "spectral_size", None)
        if NX is None:
            raise ValueError("no spectral prior set on this problem")
    if samples is None:
        samples = torch.empty((S, N), dtype=f64, device=dev)
    out = {"latent": torch.empty((S, NX), dtype=f64, device=dev) if latent and prior == "spectral" else None,
           "samples": samples,
           "mean": torch.empty(N, dtype=f64, device=dev) if stats else None,
           "std": torch.empty(N, dtype=f64, device=dev) if stats and S >= 2 else None,
           "resid": torch.empty((S, n_iter + 1), dtype=f64, device=dev) if resid else None,
           "diag": torch.empty((S, n_iter + 1, 2), dtype=f64, device=dev) if diag else None,
           "final_resid": torch.empty(S, dtype=f64, device=dev) if final else None}
    prm = RtoParams()
    prm.solver = {"cgls": PAT_CGLS, "lsqr": PAT_LSQR}[solver]
    prm.diag_hist = out["diag"].data_ptr() if diag else None
    prm.sigma = float(sigma)
    prm.prior_a = float(prior_a)
    prm.n_iter = int(n_iter)
    prm.reorth = int(bool(reorth))
    prm.sweep_prec = {"f64": PAT_F64, "f32": PAT_F32}[sweep_prec]
    prm.rhs_block = int(rhs_block)
    prm.seed = int(seed)
    prm.sample0 = int(sample0)
    prm.prior = {"fe": PAT_PRIOR_FE, "spectral": PAT_PRIOR_SPECTRAL}[prior]
    prm.latent = out["latent"].data_ptr() if out["latent"] is not None else None
    prm.final_resid = out["final_resid"].data_ptr() if final else None
    if eta is not None:
        prm.eta = _dev_ptr(eta, f64, (S, T, O), "eta")
        prm.xi = _dev_ptr(xi, f64, (S, NX), "xi")
    ptr = {"y": _dev_ptr(y_obs, f64, (T, O), "y_obs"), "samples": _dev_ptr(samples, f64, (S, N), "samples")}
    for k in ("mean", "std", "resid"):
        ptr[k] = ctypes.c_void_p(out[k].data_ptr()) if out[k] is not None else None
    return prm, S, out, ptr


def rto_sample(problem: Problem, y_obs, eta, xi, sigma: float, prior_a: float, n_iter: int, reorth: bool = True,
               sweep_prec: str = "f64", rhs_block: int = 0, stats: bool = True, resid: bool = False,
               samples=None, solver: str = "cgls", diag: bool = False, n_samples: int = None, seed: int = 0,
               sample0: int = 0, prior: str = "fe", latent: bool = False, final: bool = False):
    """RTO posterior samples (Algorithm 1) through libpat's rto_sample.

    y_obs [N_T][N_obs], eta [S][N_T][N_obs], xi [S][N]: float64 CUDA tensors.
    With eta = xi = None the library draws them itself (streams seed,
    sample0 + k; see draw_normals) and n_samples gives S.
    solver: "cgls" or "lsqr" (Sec. 5, Algorithm 1, App. A).
    prior: "fe" (the factor L with prior_a) or "spectral" (the Whittle-Matern prior set
    with spectral_prior_set; xi is then [S][n^3] and latent=True also returns the
    latent samples).
    Returns a dict with samples [S][N] and, if requested, mean, std [N],
    resid [S][n_iter+1] and diag [S][n_iter+1][2] (data and prior residual norms), and
    with final=True final_resid [S]: ||b - G_ext p|| of each sample recomputed with
    float64 sweeps after the solve."""
    prm, S, out, ptr = _rto_call(problem, y_obs, eta, xi, sigma, prior_a, n_iter, reorth, sweep_prec, rhs_block, stats,
                                 resid, samples, solver, diag, n_samples, seed, sample0, prior, latent, final)
    _check(load().rto_sample(problem._h, ptr["y"], ctypes.byref(prm), S, ptr["samples"], ptr["mean"], ptr["std"],
                             ptr["resid"], _stream()))
    return out


def autotune(problem: Problem, n_samples: int, sweep_prec: str = "f32"):
    """pat_autotune: the RHS block rto_sample(rhs_block=0) will use for n_samples; returns (block, priced us/step)."""
    rb, us = ctypes.c_int32(), ctypes.c_double()
    _check(load().pat_autotune(problem._h, int(n_samples), {"f64": PAT_F64, "f32": PAT_F32}[sweep_prec],
                               ctypes.byref(rb), ctypes.byref(us), _stream()))
    return rb.value, us.value


class Batch:
    """Handle on several problems sampled together (pat_batch_create / rto_sample_batch)."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = ctypes.c_void_p()
        self._h = None
        _check(load().pat_batch_create(arr, len(self.problems), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().pat_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def merge(self, forward: int = -1, transpose: int = -1):
        """pat_batch_merge: 1 merged launch per step, 0 one launch per problem per step,
        2 each problem's whole sweep in turn, -1 tuned."""
        _check(load().pat_batch_merge(self._h, int(forward), int(transpose)))

    def autotune(self, n_samples: int, sweep_prec: str = "f32"):
        rb, us = ctypes.c_int32(), ctypes.c_double()
        _check(load().pat_batch_autotune(self._h, int(n_samples), {"f64": PAT_F64, "f32": PAT_F32}[sweep_prec],
                                         ctypes.byref(rb), ctypes.byref(us), _stream()))
        return rb.value, us.value


def rto_sample_batch(batch: Batch, y_obs, eta, xi, sigma, prior_a, n_iter: int, reorth: bool = True,
                     sweep_prec: str = "f32", rhs_block: int = 0, stats: bool = True, resid: bool = False,
                     solver: str = "cgls", diag: bool = False, n_samples=None, seed=0, sample0=0, prior="fe",
                     final: bool = False):
    """rto_sample for every problem of the batch in one call (shared sweep launches).

    Per-problem lists: y_obs, eta, xi (entries None for device draws), sigma,
    prior_a, n_samples, seed, sample0, prior (scalars are broadcast).  Returns one
    result dict per problem."""
    n = len(batch.problems)

    def per(v):
        return list(v) if isinstance(v, (list, tuple)) else [v] * n

    eta, xi, sigma, prior_a = per(eta), per(xi), per(sigma), per(prior_a)
    n_samples, seed, sample0 = per(n_samples), per(seed), per(sample0)
    prior = [prior] * n if isinstance(prior, str) else list(prior)
    prms = (RtoParams * n)()
    S = (ctypes.c_int64 * n)()
    ys, smp, mn, sd, rs = [(ctypes.c_void_p * n)() for _ in range(5)]
    outs = []
    for m, p in enumerate(batch.problems):
        prm, S[m], out, ptr = _rto_call(p, y_obs[m], eta[m], xi[m], sigma[m], prior_a[m], n_iter, reorth, sweep_prec,
                                        rhs_block, stats, resid, None, solver, diag, n_samples[m], seed[m], sample0[m],
                                        prior[m], final=final)
        prms[m] = prm
        ys[m], smp[m] = ptr["y"].value, ptr["samples"].value
        mn[m] = ptr["mean"].value if ptr["mean"] is not None else None
        sd[m] = ptr["std"].value if ptr["std"] is not None else None
        rs[m] = ptr["resid"].value if ptr["resid"] is not None else None
        outs.append(out)
    _check(load().rto_sample_batch(batch._h, ys, prms, S, smp, mn, sd, rs, _stream()))
    return outs


def solver_diagnostics(diag, n_data: int, tau: float = 1.0):
    """Per-iteration convergence diagnostics of Sec. 6.1 (pat_solver_diagnostics) from a diag
    history [S][n_iter+1][2] of (||r_d||, ||r_p||) (float64 CUDA tensor).  Returns a dict of
    [S][n_iter+1] tensors data (||r_d|| / sqrt(n_data)), prior (||r_p|| / ||b||), extended
    (||r|| / ||b||) and "discrepancy" [S] int32: the first iteration with
    ||r_d|| <= tau sqrt(n_data), or -1."""
    import torch
    if diag.ndim != 3 or diag.shape[2] != 2:
        raise ValueError("diag must have shape [S][n_iter+1][2]")
    S, n1 = diag.shape[0], diag.shape[1]
    dp = _dev_ptr(diag, torch.float64, (S, n1, 2), "diag")
    out = {k: torch.empty((S, n1), dtype=torch.float64, device=diag.device) for k in ("data", "prior", "extended")}
    out["discrepancy"] = torch.empty(S, dtype=torch.int32, device=diag.device)
    ptr = [ctypes.c_void_p(out[k].data_ptr()) for k in ("data", "prior", "extended", "discrepancy")]
    _check(load().pat_solver_diagnostics(dp, S, n1 - 1, int(n_data), float(tau), *ptr, _stream()))
    return out


def draw_normals(seed: int, kind: int, k0: int, S: int, length: int, device="cuda"):
    """[S][length] float64 standard normals of streams (seed, kind, k0 + s), drawn on the GPU
    (Philox4x64-10 + Box-Muller); kind 0 = eta (j = t*N_obs + sensor), kind 1 = xi (j = node)."""
    import torch
    out = torch.empty((S, length), dtype=torch.float64, device=device)
    _check(load().pat_draw_normals(int(seed), int(kind), int(k0), int(S), int(length),
                                   ctypes.c_void_p(out.data_ptr()) if out.numel() else None, _stream()))
    return out


def version() -> str:
    return load().pat_version().decode()
