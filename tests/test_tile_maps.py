"""The step kernels' work mappings (which tile or sampling block each workgroup takes).

The kernels place their tiles on the XCDs with integer mappings kept in
`paper_2607_21373_amd/csrc/pat_tiles.h`: contiguous per-XCD ranges walked forward
or from their end (the transposed steps), the forward step's sampling blocks at
the front of each XCD's share, the merged multi-mesh launch, and the unequal
shares of the halo-tile kernels.  A wrong mapping would skip a tile or compute
one twice.  This test compiles a checker against that header on the host and
verifies, over tens of thousands of launch shapes (grid sizes, tile counts, mesh
sets, workgroups per XCD), that every mapping is one to one onto the tiles it
must cover and keeps the order and ranges the kernels rely on.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_21373_amd", "csrc")


def test_tile_maps(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "tile_maps_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "tile_maps_check.cpp"), "-o",
                    exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout.strip())
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
