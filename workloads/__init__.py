"""Seeded synthetic inputs for the 3D photoacoustic RTO sampler.

This module is shared by the CPU oracle (``oracle/``) and the GPU library
(``paper_2607_21373_amd``).  It holds *inputs only*: tetrahedral meshes,
per-element wave speed, sensor positions, initial-pressure phantoms and the
standard-normal draws that randomize-then-optimize consumes.  It contains none
of the method's arithmetic (no finite-element assembly, no time stepping, no
sensor interpolation, no least-squares solve), so that the two implementations
that consume these inputs stay independent.

Paper: "3D Uncertainty Quantification for Photoacoustic Tomography"
(arXiv 2607.21373).  The paper's 3D experiment (Sec. 6.4) uses an unstructured
207,151-node ball mesh that is not available; the ball meshes below are
synthetic stand-ins of the same size and geometry class.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional

import numpy as np

__all__ = [
    "kuhn_cube", "ball_mesh", "box_mesh", "cube_boundary_nodes", "fibonacci_sphere",
    "three_balls", "inclusion_3d", "uniform_ball", "smooth_bump",
    "wave_speed_bumps", "Workload", "make_workload", "rto_draws", "WORKLOADS",
]

# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

_PERMS = list(itertools.permutations(range(3)))


def _kuhn_cells(nx: int, ny: int, nz: int, mirror_centre: bool) -> np.ndarray:
    """Split an nx*ny*nz grid of cells into 6 tetrahedra per cell.

    Each cell's six tetrahedra share one main diagonal of the cell (Kuhn /
    Freudenthal split): tetrahedron ``pi`` walks from the diagonal's start
    corner along axes ``pi[0], pi[1], pi[2]``.  With ``mirror_centre`` the
    diagonal of every cell points away from the grid centre along each axis
    (cells in the lower half of an axis are reflected in that axis).  Both
    variants are conforming.  Node index = i + (nx+1)*(j + (ny+1)*k).
    """
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ii, jj, kk = ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")
    ncell = ii.size
    if mirror_centre:
        fx = (2 * ii + 1 < nx).astype(np.int64)
        fy = (2 * jj + 1 < ny).astype(np.int64)
        fz = (2 * kk + 1 < nz).astype(np.int64)
    else:
        fx = fy = fz = np.zeros(ncell, dtype=np.int64)
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    tets = np.empty((ncell, 6, 4), dtype=np.int64)
    for t, perm in enumerate(_PERMS):
        off = np.zeros((4, 3), dtype=np.int64)
        for s in range(3):
            off[s + 1] = off[s]
            off[s + 1, perm[s]] = 1
        for v in range(4):
            ox = np.where(fx == 1, 1 - off[v, 0], off[v, 0])
            oy = np.where(fy == 1, 1 - off[v, 1], off[v, 1])
            oz = np.where(fz == 1, 1 - off[v, 2], off[v, 2])
            tets[:, t, v] = (ii + ox) + sx * (jj + oy) + sy * (kk + oz)
    return tets.reshape(-1, 4)


def _orient_positive(coords: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Reorder vertices so that every tetrahedron has positive orientation."""
    neg = np.empty(tets.shape[0], dtype=bool)
    for a in range(0, tets.shape[0], 1 << 20):  # in chunks: whole-mesh temporaries are slow at 10^6 nodes
        t = tets[a:a + (1 << 20)]
        x0 = coords[t[:, 0]]
        d1, d2, d3 = coords[t[:, 1]] - x0, coords[t[:, 2]] - x0, coords[t[:, 3]] - x0
        det = np.einsum("ij,ij->i", d1, np.cross(d2, d3))
        neg[a:a + t.shape[0]] = det < 0
    tets = tets.copy()
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def box_mesh(nx: int, ny: int, nz: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             mirrored: bool = False):
    """Structured tetrahedral mesh of an axis-aligned box (6 tets per cell)."""
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    zs = np.linspace(lo[2], hi[2], nz + 1)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    coords = np.stack([X.ravel(order="F"), Y.ravel(order="F"), Z.ravel(order="F")], axis=1)
    tets = _kuhn_cells(nx, ny, nz, mirrored)
    return np.ascontiguousarray(coords), np.ascontiguousarray(_orient_positive(coords, tets).astype(np.int32))


def kuhn_cube(n: int, mirrored: bool = False):
    """Unit cube [0,1]^3 split into n^3 cells x 6 tetrahedra."""
    return box_mesh(n, n, n, mirrored=mirrored)


def ball_mesh(n: int, radius: float = 1.0):
    """Ball of the given radius from the cube [-1,1]^3 (n cells per axis).

    The cube is split with centre-mirrored Kuhn cells and mapped radially,
    x -> radius * x * |x|_inf / |x|_2, which sends the cube surface onto the
    sphere.  Mirroring keeps the mapped tetrahedra away from the degenerate
    shapes a plain Kuhn split produces near the cube's diagonals.
    """
    coords, tets = box_mesh(n, n, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), mirrored=True)
    inf = np.max(np.abs(coords), axis=1)
    two = np.linalg.norm(coords, axis=1)
    scale = np.where(two > 0, inf / np.where(two > 0, two, 1.0), 0.0)
    coords = radius * coords * scale[:, None]
    return np.ascontiguousarray(coords), np.ascontiguousarray(_orient_positive(coords, tets.astype(np.int64)).astype(np.int32))


def cube_boundary_nodes(n: int) -> np.ndarray:
    """Node ids (ascending) on the surface of the structured (n+1)^3 cube grid."""
    idx = np.arange((n + 1) ** 3)
    i, j, k = idx % (n + 1), (idx // (n + 1)) % (n + 1), idx // (n + 1) ** 2
    on = (i == 0) | (i == n) | (j == 0) | (j == n) | (k == 0) | (k == n)
    return idx[on].astype(np.int32)


def fibonacci_sphere(count: int, radius: float) -> np.ndarray:
    """Fibonacci lattice on a sphere: z_i = 1-(2i+1)/count, phi_i = i*pi*(3-sqrt 5)."""
    i = np.arange(count, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / count
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


# ---------------------------------------------------------------------------
# Phantoms (initial pressure p0 evaluated at nodes) and wave speed
# ---------------------------------------------------------------------------

def three_balls(coords: np.ndarray, seed: int = 0) -> np.ndarray:
    """Sum of three seeded indicator balls in the unit cube.

    radius ~ U(0.1, 0.2), amplitude ~ U(0.5, 1), centre ~ U([r, 1-r]^3).
    """
    rng = np.random.default_rng(seed)
    p0 = np.zeros(coords.shape[0])
    for _ in range(3):
        r = rng.uniform(0.1, 0.2)
        amp = rng.uniform(0.5, 1.0)
        centre = rng.uniform(r, 1.0 - r, size=3)
        p0 += amp * (np.linalg.norm(coords - centre, axis=1) <= r)
    return p0


def _quartic_angular(u: np.ndarray) -> np.ndarray:
    """Normalised quartic angular perturbation S(u) = 3(ux^4+uy^4+uz^4) - 2 in [-1, 1]."""
    return 3.0 * np.sum(u ** 4, axis=1) - 2.0


def inclusion_3d(coords: np.ndarray, R0: float = 0.5, alpha: float = 0.8, eps: float = 0.03,
                 centre=(0.1, 0.1, 0.1)) -> np.ndarray:
    """Smooth non-spherical inclusion of the paper's 3D experiment (Sec. 6.4).

    p0(x) = 1 / (1 + exp((|x-c| - R0 (1 + alpha S(u))) / eps)), u = (x-c)/|x-c|,
    with centre c = centre / sqrt(3).
    """
    c = np.asarray(centre, dtype=np.float64) / math.sqrt(3.0)
    d = coords - c
    r = np.linalg.norm(d, axis=1)
    u = np.where(r[:, None] > 0, d / np.where(r > 0, r, 1.0)[:, None], np.array([1.0, 0.0, 0.0]))
    arg = (r - R0 * (1.0 + alpha * _quartic_angular(u))) / eps
    return 1.0 / (1.0 + np.exp(np.clip(arg, -700.0, 700.0)))


def uniform_ball(coords: np.ndarray, R: float, amp: float = 1.0) -> np.ndarray:
    """Indicator of the ball |x| <= R times amp (nodal interpolant)."""
    return amp * (np.linalg.norm(coords, axis=1) <= R)


def smooth_bump(coords: np.ndarray, R: float, amp: float = 1.0) -> np.ndarray:
    """C^2 radial bump amp * (1 - (r/R)^2)^3 for r < R, else 0."""
    r = np.linalg.norm(coords, axis=1)
    return amp * np.where(r < R, (1.0 - (r / R) ** 2) ** 3, 0.0)


def wave_speed_bumps(coords: np.ndarray, tets: np.ndarray, seed: int = 2, amplitude: float = 0.1,
                     width: float = 0.15, n_bumps: int = 4, r_centres: float = 0.6,
                     r_taper=(0.7, 0.85)) -> np.ndarray:
    """Per-tetrahedron wave speed c = 1 + amplitude * g/max|g| * chi(r) at centroids.

    g is a sum of ``n_bumps`` seeded Gaussian bumps exp(-|x-c_b|^2/width^2) with
    random signs and centres uniform in the ball r < r_centres; chi is a cosine
    taper from 1 (r <= r_taper[0]) to 0 (r >= r_taper[1]), so c = 1 next to the
    outer boundary.
    """
    rng = np.random.default_rng(seed)
    centres = []
    while len(centres) < n_bumps:
        x = rng.uniform(-r_centres, r_centres, size=3)
        if np.linalg.norm(x) < r_centres:
            centres.append(x)
    signs = rng.choice([-1.0, 1.0], size=n_bumps)
    xc = coords[tets].mean(axis=1)
    g = np.zeros(xc.shape[0])
    for s, c in zip(signs, centres):
        g += s * np.exp(-np.sum((xc - c) ** 2, axis=1) / width ** 2)
    r = np.linalg.norm(xc, axis=1)
    a, b = r_taper
    chi = np.where(r <= a, 1.0, np.where(r >= b, 0.0, 0.5 * (1.0 + np.cos(math.pi * (r - a) / (b - a)))))
    return 1.0 + amplitude * g / np.max(np.abs(g)) * chi


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One synthetic problem: mesh, physics, sensors, truth and sampler settings.

    Exactly one of ``sensor_nodes`` (sensors at mesh nodes) and ``sensor_pos``
    (arbitrary points inside the mesh) is set.  ``noise_rule`` is "max" for
    sigma = d_noise * max|Y| or "l2" for the paper's relative-L2 rule.
    """
    name: str
    coords: np.ndarray
    tets: np.ndarray
    c_tet: Optional[np.ndarray]
    absorbing: bool
    dt: float
    n_steps: int
    sensor_nodes: Optional[np.ndarray] = None
    sensor_pos: Optional[np.ndarray] = None
    p0_true: Optional[np.ndarray] = None
    d_noise: float = 0.01
    noise_rule: str = "l2"
    noise_seed: int = 3
    prior_a: float = 0.01
    n_samples: int = 16
    n_iter: int = 100
    rto_seed: int = 1
    h: float = 0.0

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.sensor_nodes.size if self.sensor_nodes is not None else self.sensor_pos.shape[0])


def _cube_tiny() -> Workload:
    n = 8
    coords, tets = kuhn_cube(n)
    h = 1.0 / n
    bnodes = cube_boundary_nodes(n)
    return Workload(
        name="cube8_tiny", coords=coords, tets=tets, c_tet=None, absorbing=False,
        dt=0.3 * h, n_steps=200, sensor_nodes=bnodes[::6][:64].copy(),
        p0_true=three_balls(coords, seed=0), noise_rule="max", noise_seed=3,
        prior_a=0.01, n_samples=10, n_iter=50, rto_seed=1, h=h)


def _ball(n_cells: int, n_sensors: int, n_steps: int, name: str, n_samples: int,
          rto_seed: int, variable_c: bool = True) -> Workload:
    coords, tets = ball_mesh(n_cells)
    h = 2.0 / n_cells
    c = wave_speed_bumps(coords, tets, seed=2) if variable_c else None
    return Workload(
        name=name, coords=coords, tets=tets, c_tet=c, absorbing=True,
        dt=0.2 * h, n_steps=n_steps, sensor_pos=fibonacci_sphere(n_sensors, 0.9),
        p0_true=inclusion_3d(coords, R0=0.25, alpha=0.8, eps=0.015, centre=(0.05, 0.05, 0.05)),
        noise_rule="l2", noise_seed=3, prior_a=0.01, n_samples=n_samples, n_iter=100,
        rto_seed=rto_seed, h=h)


def _top_face_grid(nx: int, ny: int, nz: int, gx: int = 32, gy: int = 16) -> np.ndarray:
    """gx x gy node sensors (at most the face) centred on the top face z = max of an (nx+1)(ny+1)(nz+1) grid."""
    gx, gy = min(gx, nx + 1), min(gy, ny + 1)
    i0, j0 = (nx + 1 - gx) // 2, (ny + 1 - gy) // 2
    i, j = np.meshgrid(np.arange(i0, i0 + gx), np.arange(j0, j0 + gy), indexing="ij")
    k = nz
    return (i.ravel() + (nx + 1) * (j.ravel() + (ny + 1) * k)).astype(np.int32)


def _box(name: str, nx: int, ny: int, nz: int, n_samples: int = 16, rto_seed: int = 11) -> Workload:
    """Absorbing box [0,1] x [0,1] x [0, nz/nx] with cubic cells of side h = 1/nx."""
    h = 1.0 / nx
    coords, tets = box_mesh(nx, ny, nz, hi=(1.0, ny * h, nz * h), mirrored=True)
    depth = nz * h
    centre = np.array([0.5, 0.5 * ny * h, 0.5 * depth])
    rng = np.random.default_rng(13)
    p0 = np.zeros(coords.shape[0])
    for _ in range(3):                       # three smooth bumps inside the box
        R = 0.4 * min(depth, 0.5) * rng.uniform(0.6, 1.0)
        c = centre + rng.uniform(-0.25, 0.25, size=3) * np.array([1.0, 1.0, depth - 2 * R])
        p0 += rng.uniform(0.5, 1.0) * smooth_bump(coords - c, R)
    return Workload(name=name, coords=coords, tets=tets, c_tet=None, absorbing=True, dt=0.2 * h, n_steps=1000,
                    sensor_nodes=_top_face_grid(nx, ny, nz), p0_true=p0, noise_rule="l2", noise_seed=3,
                    prior_a=0.01, n_samples=n_samples, n_iter=100, rto_seed=rto_seed, h=h)


def make_workload(name: str) -> Workload:
    """Build a named workload.

    * ``cube8_tiny``: unit cube, 8^3 cells, 729 nodes, reflecting, dt = 0.3h,
      200 steps, 64 node sensors on the surface, 10 samples x 50 iterations.
    * ``ball58_fp64``: 58^3-node mapped ball (195,112 nodes), variable c,
      absorbing, dt = 0.2h, 1000 steps, 1024 sensors on r = 0.9, 16 samples
      x 100 iterations.
    * ``ball58_batched``: same problem, 64 samples (one multi-RHS batch).
    * ``ball16``: 17^3-node ball with the same recipe (for fast parity tests),
      200 steps, 64 sensors.
    * ``cube40``, ``ball60``, ``slab120``: the uneven three-mesh batch: 40^3-node
      cube, 60^3-node ball, 120 x 120 x 30-node slab; absorbing, dt = 0.2h,
      1000 steps, 512 sensors (a 32 x 16 node grid on the top face of the cube
      and the slab, a Fibonacci lattice on r = 0.9 for the ball), 16 samples each.
    * ``ball100``: 100^3-node ball (10^6 nodes) with the ball58 recipe, one sample.
    * ``box12``: 12 x 12 x 6-node absorbing box, 200 steps (a small uneven-batch member).
    """
    if name == "cube8_tiny":
        return _cube_tiny()
    if name == "ball58_fp64":
        return _ball(57, 1024, 1000, name, n_samples=16, rto_seed=5)
    if name == "ball58_batched":
        return _ball(57, 1024, 1000, name, n_samples=64, rto_seed=5)
    if name == "ball16":
        w = _ball(16, 64, 200, name, n_samples=16, rto_seed=7)
        w.n_iter = 50
        return w
    if name == "box12":
        w = _box(name, 11, 11, 5, rto_seed=21)
        w.n_steps = 200
        w.n_iter = 30
        return w
    if name == "cube40":
        return _box(name, 39, 39, 39, rto_seed=11)
    if name == "slab120":
        return _box(name, 119, 119, 29, rto_seed=12)
    if name == "ball60":
        return _ball(59, 512, 1000, name, n_samples=16, rto_seed=13)
    if name == "ball100":
        return _ball(99, 1024, 1000, name, n_samples=1, rto_seed=14)
    raise KeyError(name)


WORKLOADS = ("cube8_tiny", "ball58_fp64", "ball58_batched", "ball16", "box12", "cube40", "ball60", "slab120",
             "ball100")


def rto_draws(n_samples: int, n_steps: int, n_obs: int, n_nodes: int, seed: int):
    """Standard-normal RTO perturbations: eta [S][n_steps][n_obs], xi [S][n_nodes]."""
    rng = np.random.default_rng(seed)
    eta = rng.standard_normal((n_samples, n_steps, n_obs))
    xi = rng.standard_normal((n_samples, n_nodes))
    return eta, xi


def noise_draw(n_steps: int, n_obs: int, seed: int) -> np.ndarray:
    """Standard-normal data-noise realization eta0 [n_steps][n_obs]."""
    return np.random.default_rng(seed).standard_normal((n_steps, n_obs))
