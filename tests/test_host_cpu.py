"""CPU checks of libpat's host side: exports, setup parity with the oracle, error paths.

None of these launch a kernel: pat_problem_create validates and assembles on the
host before it touches a device, and pat_host_assemble stops before the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

pat = pytest.importorskip("paper_2607_21373_amd.pat")
from paper_2607_21373_amd.pat import PatError  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "pat.h")).read()
    declared = set(re.findall(r"^\s*(?:pat_status|const char \*)\s*(\w+)\s*\(", header, re.M))
    assert {"pat_forward", "pat_adjoint", "rto_sample", "pat_problem_create"} <= declared
    lib = ctypes.CDLL(pat.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert set(pat.EXPORTS) == declared
    assert "gfx950" in pat.version()


def _csr_dense(rowptr, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rowptr[i]:rowptr[i + 1]]] = val[rowptr[i]:rowptr[i + 1]]
    return A


@pytest.mark.parametrize("case", ["cube8", "ball6_varc", "ball16"])
def test_host_assembly_matches_oracle(case):
    if case == "cube8":
        w = W.make_workload("cube8_tiny")
        args = dict(coords=w.coords, tets=w.tets, c_tet=None, absorbing=False, dt=w.dt, n_steps=5,
                    sensor_nodes=w.sensor_nodes)
    elif case == "ball6_varc":
        coords, tets = W.ball_mesh(6)
        c = W.wave_speed_bumps(coords, tets, seed=2, r_taper=(0.4, 0.7), r_centres=0.4)
        args = dict(coords=coords, tets=tets, c_tet=c, absorbing=True, dt=0.05, n_steps=5,
                    sensor_pos=W.fibonacci_sphere(40, 0.8))
    else:
        w = W.make_workload("ball16")
        args = dict(coords=w.coords, tets=w.tets, c_tet=w.c_tet, absorbing=True, dt=w.dt, n_steps=5,
                    sensor_pos=w.sensor_pos)
    h = pat.pat_host_assemble(**args)
    P = oracle.Problem(**args)
    n = P.n_nodes
    for name, key in (("K", "K"), ("K1", "K1"), ("B", "B")):
        ref = P.matrix(name)
        got = _csr_dense(h["rowptr"], h["col"], h[key], n) if n < 1000 else None
        if got is not None:
            scale = np.abs(ref.toarray()).max() if ref.nnz else 1.0
            assert np.abs(got - ref.toarray()).max() <= 1e-13 * scale, name
        else:
            import scipy.sparse as sp
            A = sp.csr_matrix((h[key], h["col"], h["rowptr"]), shape=(n, n))
            scale = abs(ref).max() if ref.nnz else 1.0
            assert abs(A - ref).max() <= 1e-13 * scale, name
    np.testing.assert_allclose(h["mass"], P.lumped_mass(), rtol=1e-13)
    on, ow = P.sensors()
    # same interpolant: weights agree node by node
    for s in range(P.n_obs):
        a = dict()
        for k in range(4):
            a[on[s, k]] = a.get(on[s, k], 0.0) + ow[s, k]
        b = dict()
        for k in range(4):
            b[h["snode"][s, k]] = b.get(h["snode"][s, k], 0.0) + h["sw"][s, k]
        for key in set(a) | set(b):
            assert abs(a.get(key, 0.0) - b.get(key, 0.0)) < 1e-12


def test_lambda_max_estimate():
    import scipy.sparse.linalg as sla
    w = W.make_workload("ball16")
    h = pat.pat_host_assemble(w.coords, w.tets, w.c_tet, True, w.dt, 5, sensor_pos=w.sensor_pos)
    P = oracle.Problem.from_workload(w, n_steps=5)
    m = P.lumped_mass()
    import scipy.sparse as sp
    D = sp.diags(1 / np.sqrt(m))
    lam = sla.eigsh(D @ P.matrix("K") @ D, k=1, which="LA", return_eigenvectors=False)[0]
    assert 0.98 * lam <= h["lambda_max"] <= 1.0000001 * lam


def _tiny():
    coords, tets = W.ball_mesh(4)
    return dict(coords=coords, tets=tets, c_tet=None, absorbing=True, dt=0.05, n_steps=10,
                sensor_pos=W.fibonacci_sphere(8, 0.7))


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a.update(dt=-1.0), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(dt=float("nan")), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(n_steps=0), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(tets=np.where(a["tets"] == 3, 10 ** 6, a["tets"])), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(c_tet=np.full(a["tets"].shape[0], -1.0)), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(sensor_pos=np.array([[3.0, 0.0, 0.0]])), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(sensor_nodes=np.array([0, 1], np.int32)), "PAT_ERR_INVALID_ARG"),   # both kinds given
    (lambda a: (a.pop("sensor_pos"), a.update(sensor_nodes=np.array([999], np.int32))), "PAT_ERR_INVALID_ARG"),
    (lambda a: a["coords"].__setitem__((0, 0), np.inf), "PAT_ERR_NONFINITE"),
    (lambda a: a.update(tets=np.vstack([a["tets"], [[0, 0, 1, 2]]]).astype(np.int32)), "PAT_ERR_INVALID_ARG"),
    (lambda a: a.update(dt=1.0), "PAT_ERR_UNSTABLE_DT"),
])
def test_create_rejects_bad_input(mutate, code):
    a = _tiny()
    a["coords"] = a["coords"].copy()
    mutate(a)
    with pytest.raises(PatError) as ei:
        pat.Problem(**a)
    assert ei.value.name == code, str(ei.value)
    with pytest.raises(PatError) as ei2:
        pat.pat_host_assemble(**a)
    assert ei2.value.name == code


def test_explicit_boundary_term_instability_detected():
    """dt inside the B = 0 CFL bound but too large for the explicit absorbing term."""
    coords, tets = W.kuhn_cube(6)          # plain Kuhn split: large boundary-to-mass ratios at corners
    h = 1.0 / 6
    base = dict(coords=coords, tets=tets, n_steps=5, sensor_nodes=np.array([0], np.int32))
    lam = pat.pat_host_assemble(dt=0.1 * h, absorbing=True, **base)["lambda_max"]
    dt = 0.95 * 2 / np.sqrt(lam)           # dt^2 lambda = 3.6 < 4
    pat.pat_host_assemble(dt=dt, absorbing=False, **base)
    with pytest.raises(PatError) as ei:
        pat.pat_host_assemble(dt=dt, absorbing=True, **base)
    assert ei.value.name == "PAT_ERR_UNSTABLE_DT"


def test_create_without_device_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(PatError) as ei:
        pat.Problem(**_tiny())
    assert ei.value.name == "PAT_ERR_HIP"


def test_binding_structs_match_header(tmp_path):
    """Field offsets and sizes of the ctypes structs equal those gcc computes from include/pat.h."""
    import subprocess
    structs = {"pat_problem_desc": pat.ProblemDesc, "pat_problem_info": pat.ProblemInfo,
               "pat_rto_params": pat.RtoParams, "pat_profile": pat.Profile, "pat_spectral_desc": pat.SpectralDesc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pat.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = structs[cname]
        got = ctypes.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


def test_solver_diagnostics_on_oracle_histories():
    """The oracle's diagnostics of Sec. 6.1: discrepancy principle on the whitened data residual of
    the MAP solve (eta = xi = 0); the extended residual is the carried LSQR residual, normalised."""
    w = W.make_workload("cube8_tiny")
    O = oracle.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    M = w.n_steps * w.n_obs
    zeros_d = np.zeros((1, w.n_steps, w.n_obs))
    x, res, dg = O.lsqr(yobs[None] / sigma + zeros_d, np.zeros((1, w.n_nodes)), sigma, w.prior_a, 30, diag=True)
    out = oracle.diagnostics(dg, M)
    np.testing.assert_allclose(out["extended"][0], res[0] / res[0, 0], rtol=1e-14)
    assert out["extended"][0, 0] == 1.0 and out["prior"][0, 0] == 0.0
    # the LSQR residual of the extended system is non-increasing
    assert np.all(np.diff(res[0]) <= 1e-12 * res[0, 0])
    k = int(out["discrepancy"][0])
    assert k >= 1 and out["data"][0, k] <= 1.0 and np.all(out["data"][0, :k] > 1.0)
    # tau large enough: satisfied at iteration 0; tau tiny: never
    assert oracle.diagnostics(dg, M, tau=1e9)["discrepancy"][0] == 0
    assert oracle.diagnostics(dg, M, tau=1e-9)["discrepancy"][0] == -1
    with pytest.raises(ValueError):
        oracle.diagnostics(dg[..., 0], M)
