"""The halo tiles of the float32 step kernels (host setup) against their definition.

The halo step kernels copy, per tile of consecutive rows, the distinct
neighbour rows the tile's padded slots refer to into LDS and read every slot
from there (Sec. 3 eq. (discrete-wave-matrix) applied row by row).  This test
compiles a small checker against the library's host setup and verifies, on
several meshes, that the tiles partition the rows in order, that each halo is
exactly the sorted set of referenced rows, that every slot's local index names
its column, and that the metadata words hold the padded layout's operands.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_21373_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("halo") / "halo_tiles_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "halo_tiles_check.cpp"), os.path.join(CSRC, "pat_setup.cpp"), "-o",
                    out], check=True)
    return out


def _dump(w, path):
    with open(path, "wb") as f:
        E = w.tets.shape[0]
        f.write(np.int32(w.n_nodes).tobytes())
        f.write(np.int64(E).tobytes())
        f.write(np.ascontiguousarray(w.coords, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(w.tets, dtype=np.int32).tobytes())
        c = w.c_tet if w.c_tet is not None else np.ones(E)
        f.write(np.ascontiguousarray(c, dtype=np.float64).tobytes())
        sp = w.sensor_pos if w.sensor_pos is not None else w.coords[w.sensor_nodes]
        f.write(np.int32(sp.shape[0]).tobytes())
        f.write(np.ascontiguousarray(sp, dtype=np.float64).tobytes())
        f.write(np.float64(w.dt).tobytes())
        f.write(np.int32(w.n_steps).tobytes())


@pytest.mark.parametrize("name", ["cube8_tiny", "ball16", "box12", "cube40"])
def test_halo_tiles(checker, tmp_path, name):
    w = W.make_workload(name)
    path = str(tmp_path / f"{name}.bin")
    _dump(w, path)
    r = subprocess.run([checker, path], capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
