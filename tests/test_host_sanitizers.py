"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* libpat's host setup (pat_setup.cpp, built with g++ and the sanitizers into a
  small driver) on valid meshes and on invalid inputs, each of which must end
  in its documented pat_status with no sanitizer report;
* the oracle (pat_oracle.c, built with gcc and the sanitizers) running forward,
  transpose, CGLS/LSQR RTO and the normal draws in a child process that
  preloads the sanitizer runtimes.
Any sanitizer finding aborts the child process, which fails the test.
"""
import os
import shutil
import struct
import subprocess
import sys

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-O1", "-g"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


pytestmark = pytest.mark.skipif(shutil.which("g++") is None or _runtime("libasan.so") is None,
                                reason="g++ with the ASan runtime is needed")


def _dump(path, w, dt=None, sensor_nodes=None, sensor_pos=None, tets=None):
    sn = w.sensor_nodes if sensor_nodes is None else sensor_nodes
    sp = w.sensor_pos if sensor_pos is None else sensor_pos
    mode = 1 if (sp is not None and sensor_nodes is None) else 0
    T = w.tets if tets is None else tets
    has_c = w.c_tet is not None
    with open(path, "wb") as f:
        f.write(struct.pack("7i", w.n_nodes, len(T), sp.shape[0] if mode else sn.size, int(has_c), mode,
                            int(w.absorbing), w.n_steps))
        f.write(struct.pack("d", w.dt if dt is None else dt))
        f.write(np.ascontiguousarray(w.coords, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(T, dtype=np.int32).tobytes())
        if has_c:
            f.write(np.ascontiguousarray(w.c_tet, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(sp, dtype=np.float64).tobytes() if mode
                else np.ascontiguousarray(sn, dtype=np.int32).tobytes())


def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_setup_driver")
    subprocess.run(["g++", "-std=c++17", "-pthread", *SAN, "-I", os.path.join(ROOT, "paper_2607_21373_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "host_setup_driver.cpp"),
                    os.path.join(ROOT, "paper_2607_21373_amd", "csrc", "pat_setup.cpp"), "-o", exe], check=True)
    cube, ball = W.make_workload("cube8_tiny"), W.make_workload("ball16")
    cases = {"cube8_tiny": (cube, {}, 0, "status 0"), "ball16": (ball, {}, 0, "status 0"),
             "box12": (W.make_workload("box12"), {}, 0, "status 0")}
    sp = ball.sensor_pos.copy()
    sp[3] = (5.0, 0.0, 0.0)
    sn = cube.sensor_nodes.copy()
    sn[0] = cube.n_nodes
    T = cube.tets.copy()
    T[5, 2] = -1
    cases.update({"unstable_dt": (ball, {"dt": 10 * ball.dt}, 1, "status -2"),
                  "sensor_outside": (ball, {"sensor_pos": sp}, 1, "status -1"),
                  "sensor_node_range": (cube, {"sensor_nodes": sn}, 1, "status -1"),
                  "tet_node_range": (cube, {"tets": T}, 1, "status -1")})
    for name, (w, kw, code, text) in cases.items():
        path = str(tmp_path / f"{name}.bin")
        _dump(path, w, **kw)
        r = subprocess.run([exe, path], capture_output=True, text=True, timeout=300)
        print(name, r.returncode, r.stdout.strip(), r.stderr[-300:])
        assert r.returncode == code and text in r.stdout, (name, r.stdout, r.stderr[-2000:])


ORACLE_RUN = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[2])
import oracle, workloads as W
oracle._LIB = sys.argv[1]
for name in ("cube8_tiny", "ball16"):
    w = W.make_workload(name)
    O = oracle.Problem.from_workload(w)
    Y, yobs, sigma = oracle.synthesize(O, w)
    p = np.random.default_rng(0).standard_normal((3, w.n_nodes))
    y = O.forward(p)
    a = O.adjoint(y)
    eta, xi = W.rto_draws(4, w.n_steps, w.n_obs, w.n_nodes, w.rto_seed)
    for solver in ("cgls", "lsqr"):
        O.rto(yobs, sigma, w.prior_a, 6, eta, xi, solver=solver)
    oracle.normals(3, 0, 0, 2, 1000)
print("oracle ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", *SAN, "-o", lib,
                    os.path.join(ROOT, "oracle", "pat_oracle.c"), "-lm"], check=True)
    pre = " ".join(p for p in (_runtime("libasan.so"), _runtime("libubsan.so")) if p)
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", ORACLE_RUN, lib, ROOT], capture_output=True, text=True, timeout=900,
                       env=env)
    print(r.stdout[-500:], r.stderr[-3000:])
    assert r.returncode == 0 and "oracle ok" in r.stdout
