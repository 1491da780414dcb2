"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: closed
forms (7-point stencil of the Kuhn split, boundary integrals of linear
functions, d'Alembert's radial solution), exact invariants of the Stormer-Verlet
step (discrete energy), the paper's block-matrix and factored forms of the
propagator, dense transposes, Krylov-space minimisers and the exact posterior
of App. A.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import _dense


def _tiny_ball(n=4, n_steps=20, n_sens=8, absorbing=True, variable_c=True):
    coords, tets = W.ball_mesh(n)
    c = W.wave_speed_bumps(coords, tets, seed=2, r_taper=(0.3, 0.6), r_centres=0.3) if variable_c else None
    h = 2.0 / n
    P = oracle.Problem(coords, tets, c, absorbing, 0.2 * h, n_steps, sensor_pos=W.fibonacci_sphere(n_sens, 0.7))
    return P, coords, tets, c


@pytest.fixture(scope="module")
def cube8():
    w = W.make_workload("cube8_tiny")
    return w, oracle.Problem.from_workload(w)


@pytest.fixture(scope="module")
def tiny():
    return _tiny_ball()


def _faces_numpy(tets):
    """Boundary faces (node triples) by counting sorted face keys with numpy."""
    f = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    fs = np.sort(f, axis=1)
    u, idx, cnt = np.unique(fs, axis=0, return_index=True, return_counts=True)
    return f[idx[cnt == 1]]


# ---------------------------------------------------------------------------
# Assembly (Sec. 3, matrices under eq. (semi-discrete); lumped mass)
# ---------------------------------------------------------------------------

def test_kuhn_cube_interior_stencil(cube8):
    """On the Kuhn-split cube with c = 1, interior rows of K are h*(6, -1 x 6) and M_L = h^3."""
    w, P = cube8
    n = 8
    h = 1.0 / n
    K = P.matrix("K").toarray()
    m = P.lumped_mass()
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                row = i + (n + 1) * (j + (n + 1) * k)
                expect = np.zeros(K.shape[0])
                expect[row] = 6 * h
                for d in (1, n + 1, (n + 1) ** 2):
                    expect[row + d] = expect[row - d] = -h
                np.testing.assert_allclose(K[row], expect, atol=1e-15)
                assert abs(m[row] - h ** 3) < 1e-17


def test_constant_speed_scales_stiffness():
    """K scales with c^2 and B with 1/c for a constant speed c."""
    coords, tets = W.ball_mesh(4)
    h = 0.5
    P1 = oracle.Problem(coords, tets, None, True, 0.1 * h, 2, sensor_nodes=[0])
    P2 = oracle.Problem(coords, tets, np.full(tets.shape[0], 1.5), True, 0.1 * h, 2, sensor_nodes=[0])
    np.testing.assert_allclose(P2.matrix("K").toarray(), 2.25 * P1.matrix("K").toarray(), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(P2.matrix("B").toarray(), P1.matrix("B").toarray() / 1.5, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(P2.matrix("K1").toarray(), P1.matrix("K").toarray(), rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("mesh", ["cube", "ball"])
def test_stiffness_identities(mesh):
    """K 1 = 0, K symmetric PSD, and u^T K u = |a|^2 vol for linear u = a.x (c = 1)."""
    if mesh == "cube":
        coords, tets = W.kuhn_cube(5, mirrored=True)
    else:
        coords, tets = W.ball_mesh(6)
    P = oracle.Problem(coords, tets, None, True, 0.01, 2, sensor_nodes=[0])
    K = P.matrix("K").toarray()
    m = P.lumped_mass()
    assert np.abs(K.sum(axis=1)).max() < 1e-14
    assert np.abs(K - K.T).max() < 1e-16
    assert np.linalg.eigvalsh(K).min() > -1e-13
    vol = _volume_divergence(coords, tets)
    assert abs(m.sum() - vol) < 1e-13 * vol
    a = np.array([0.3, -1.2, 0.7])
    u = coords @ a
    assert abs(u @ K @ u - a @ a * vol) < 1e-12 * vol


def _volume_divergence(coords, tets):
    """Polyhedron volume from its boundary faces, V = (1/3) sum over faces of x . n dA."""
    faces = _faces_numpy(tets)
    # orient each face outward using the centroid of its own tetrahedron's opposite vertex
    f = np.sort(faces, axis=1)
    allf = np.concatenate([np.sort(tets[:, [1, 2, 3]], axis=1), np.sort(tets[:, [0, 2, 3]], axis=1),
                           np.sort(tets[:, [0, 1, 3]], axis=1), np.sort(tets[:, [0, 1, 2]], axis=1)])
    opp = np.concatenate([tets[:, 0], tets[:, 1], tets[:, 2], tets[:, 3]])
    key = {tuple(k): o for k, o in zip(map(tuple, allf), opp)}
    vol = 0.0
    for tri in f:
        x0, x1, x2 = coords[tri[0]], coords[tri[1]], coords[tri[2]]
        nrm = np.cross(x1 - x0, x2 - x0)
        if np.dot(nrm, x0 - coords[key[tuple(tri)]]) < 0:
            nrm = -nrm
        vol += np.dot(x0, nrm) / 6.0
    return vol


def test_boundary_mass_cube_closed_form():
    """1^T B 1 = area(boundary) = 6 and x^T B x = int_boundary x^2 dS = 7/3 on the unit cube."""
    coords, tets = W.kuhn_cube(4)
    P = oracle.Problem(coords, tets, None, True, 0.01, 2, sensor_nodes=[0])
    B = P.matrix("B").toarray()
    one = np.ones(coords.shape[0])
    assert abs(one @ B @ one - 6.0) < 1e-13
    x = coords[:, 0]
    assert abs(x @ B @ x - 7.0 / 3.0) < 1e-13
    xy = coords[:, 0] + 2 * coords[:, 1]
    # int over the cube surface of (x + 2y)^2: faces x=0,1: int (x+2y)^2 dy dz ; y=0,1 ; z=0,1
    exact = (4.0 / 3.0) + (1 + 2 + 4.0 / 3.0) + (1.0 / 3.0) + (1.0 / 3.0 + 2 + 4) + 2 * (1.0 / 3.0 + 1 + 4.0 / 3.0)
    assert abs(xy @ B @ xy - exact) < 1e-12
    interior = np.ones(coords.shape[0], bool)
    interior[W.cube_boundary_nodes(4)] = False
    assert np.abs(B[interior]).max() == 0.0
    assert np.linalg.eigvalsh(B).min() > -1e-15


def test_boundary_mass_ball_area():
    """1^T B 1 equals the polyhedral surface area (independent face count) and tends to 4 pi."""
    coords, tets = W.ball_mesh(16)
    P = oracle.Problem(coords, tets, None, True, 0.01, 2, sensor_nodes=[0])
    faces = _faces_numpy(tets)
    area = 0.5 * np.linalg.norm(np.cross(coords[faces[:, 1]] - coords[faces[:, 0]],
                                         coords[faces[:, 2]] - coords[faces[:, 0]]), axis=1).sum()
    B = P.matrix("B")
    assert abs(B.sum() - area) < 1e-12 * area
    assert abs(area - 4 * math.pi) < 0.005 * 4 * math.pi
    Pr = oracle.Problem(coords, tets, None, False, 0.01, 2, sensor_nodes=[0])
    assert Pr.matrix("B").nnz == 0


def test_sensor_interpolation_reproduces_linear():
    """Barycentric Pi reproduces linear functions at the sensor points; weights sum to 1."""
    coords, tets = W.ball_mesh(8)
    pts = W.fibonacci_sphere(50, 0.9)
    P = oracle.Problem(coords, tets, None, True, 0.01, 2, sensor_pos=pts)
    nodes, wts = P.sensors()
    assert np.all(wts > -1e-12)
    np.testing.assert_allclose(wts.sum(axis=1), 1.0, atol=1e-14)
    recon = np.einsum("sk,skd->sd", wts, coords[nodes])
    np.testing.assert_allclose(recon, pts, atol=1e-14)
    with pytest.raises(ValueError):
        oracle.Problem(coords, tets, None, True, 0.01, 2, sensor_pos=np.array([[2.0, 0.0, 0.0]]))


# ---------------------------------------------------------------------------
# Forward step and forward map (Sec. 3 eqs. (fully-discrete), (matrix-stromer),
# (discrete-wave-matrix); App. B)
# ---------------------------------------------------------------------------

def test_step_matches_block_propagator(tiny):
    P = tiny[0]
    K, B, m = P.matrix("K").toarray(), P.matrix("B").toarray(), P.lumped_mass()
    A = _dense.propagator_block(K, B, m, P.dt)
    S1, S2, S3, S4 = _dense.propagator_factors(K, B, m, P.dt)
    np.testing.assert_allclose(S4 @ S3 @ S2 @ S1, A, atol=1e-14)
    N = P.n_nodes
    rng = np.random.default_rng(0)
    p, v = rng.standard_normal((3, N)), rng.standard_normal((3, N))
    pn, vn = P.step(p, v)
    z = A @ np.hstack([p, v]).T
    np.testing.assert_allclose(np.hstack([pn, vn]).T, z, rtol=0, atol=1e-13 * np.abs(z).max())


def test_transpose_step_matches_block_transpose(tiny):
    P = tiny[0]
    K, B, m = P.matrix("K").toarray(), P.matrix("B").toarray(), P.lumped_mass()
    A = _dense.propagator_block(K, B, m, P.dt)
    S1, S2, S3, S4 = _dense.propagator_factors(K, B, m, P.dt)
    np.testing.assert_allclose(S1.T @ S2.T @ S3.T @ S4.T, A.T, atol=1e-14)
    N = P.n_nodes
    rng = np.random.default_rng(1)
    ph, vh = rng.standard_normal((2, N)), rng.standard_normal((2, N))
    a, b = P.step_transpose(ph, vh)
    z = A.T @ np.hstack([ph, vh]).T
    np.testing.assert_allclose(np.hstack([a, b]).T, z, rtol=0, atol=1e-13 * np.abs(z).max())


def test_forward_map_matches_dense_powers(tiny):
    P = tiny[0]
    K, B, m = P.matrix("K").toarray(), P.matrix("B").toarray(), P.lumped_mass()
    A = _dense.propagator_block(K, B, m, P.dt)
    nodes, wts = P.sensors()
    Pi = _dense.sensor_matrix(nodes, wts, P.n_nodes)
    G = _dense.forward_matrix(A, Pi, P.n_steps)
    cols = P.forward(np.eye(P.n_nodes))                     # [N][N_T][N_obs]: column i = G e_i
    Gor = cols.reshape(P.n_nodes, -1).T
    np.testing.assert_allclose(Gor, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_dense_transpose(tiny):
    """G^T assembled column by column from the backward recursion equals (G)^T."""
    P = tiny[0]
    N, M = P.n_nodes, P.n_steps * P.n_obs
    G = P.forward(np.eye(N)).reshape(N, -1).T
    GT = P.adjoint(np.eye(M).reshape(M, P.n_steps, P.n_obs))   # row j = G^T e_j
    np.testing.assert_allclose(GT, G, rtol=0, atol=1e-13 * np.abs(G).max())


@pytest.mark.parametrize("name", ["cube8_tiny", "ball16"])
def test_transpose_identity(name):
    """<G p, yhat> = <p, G^T yhat> to 1e-13 relative (Sec. 6.1)."""
    w = W.make_workload(name)
    P = oracle.Problem.from_workload(w)
    rng = np.random.default_rng(4)
    p = rng.standard_normal((2, P.n_nodes))
    yh = rng.standard_normal((2, P.n_steps, P.n_obs))
    lhs = np.einsum("rts,rts->r", P.forward(p), yh)
    rhs = np.einsum("rn,rn->r", p, P.adjoint(yh))
    assert np.all(np.abs(lhs - rhs) <= 1e-13 * np.abs(lhs))


def _energy(K, m, p, v, dt):
    return 0.5 * np.sum(m * v * v) + 0.5 * p @ (K @ p) - dt ** 2 / 8 * v @ (K @ v)


def test_energy_conserved_without_absorption(cube8):
    """B = 0: E = v'M_L v/2 + p'Kp/2 - dt^2 v'Kv/8 is invariant under the step."""
    w, P = cube8
    K, m = P.matrix("K"), P.lumped_mass()
    p, v = w.p0_true.copy(), np.zeros(P.n_nodes)
    e0 = _energy(K, m, p, v, P.dt)
    for _ in range(200):
        p, v = (a[0] for a in P.step(p, v))
        assert abs(_energy(K, m, p, v, P.dt) - e0) < 1e-13 * e0


def test_energy_balance_with_absorption():
    """With B: E^{n+1} - E^n = -(dt/2) v^n' B (v^n + v^{n+1}) exactly; energy decays."""
    coords, tets = W.ball_mesh(8)
    h = 0.25
    P = oracle.Problem(coords, tets, None, True, 0.2 * h, 2, sensor_nodes=[0])
    K, B, m = P.matrix("K"), P.matrix("B"), P.lumped_mass()
    p, v = W.smooth_bump(coords, 0.6), np.zeros(P.n_nodes)
    e = _energy(K, m, p, v, P.dt)
    e_first = e
    for _ in range(150):
        pn, vn = (a[0] for a in P.step(p, v))
        en = _energy(K, m, pn, vn, P.dt)
        expect = -(P.dt / 2) * v @ (B @ (v + vn))
        assert abs((en - e) - expect) < 1e-13 * e_first
        p, v, e = pn, vn, en
    assert e < 0.5 * e_first


def test_radial_bump_second_order():
    """Smooth radial p0: sensor traces converge to d'Alembert's p = [(r-t)p0(|r-t|)+(r+t)p0(r+t)]/(2r)."""
    errs = []
    R, r = 0.3, 0.5
    f = lambda s: np.where(np.abs(s) < R, (1 - (s / R) ** 2) ** 3, 0.0)
    for n in (16, 32):
        coords, tets = W.ball_mesh(n)
        h = 2.0 / n
        dt = 0.2 * h
        nt = int(round(0.85 / dt))
        sens = np.array([[r, 0, 0], [0, -r, 0], [0, 0, r]])
        P = oracle.Problem(coords, tets, None, True, dt, nt, sensor_pos=sens)
        t = dt * np.arange(1, nt + 1)
        y = P.forward(W.smooth_bump(coords, R))
        ex = ((r - t) * f(np.abs(r - t)) + (r + t) * f(r + t)) / (2 * r)
        errs.append(np.sqrt(np.mean((y - ex[:, None]) ** 2)) / np.sqrt(np.mean(ex ** 2)))
    assert errs[1] < 0.4 * errs[0]          # at least ~1.3 order from h to h/2
    assert errs[1] < 0.3


def test_uniform_ball_n_wave():
    """Uniform ball of initial pressure: N-wave A(r-t)/(2r) for |r-t| < R at a sensor at radius r.

    The nodal indicator has effective radius R_eff = (3 sum M_L p0 / 4pi)^(1/3); the
    time-integrated trace converges to that of the closed form under refinement."""
    R, r = 0.3, 0.5
    errs = []
    for n in (16, 48):
        coords, tets = W.ball_mesh(n)
        h = 2.0 / n
        dt = 0.2 * h
        nt = int(round(0.85 / dt))
        P = oracle.Problem(coords, tets, None, True, dt, nt, sensor_pos=np.array([[r, 0, 0], [0, 0, -r]]))
        p0 = W.uniform_ball(coords, R)
        Reff = (3 * np.sum(P.lumped_mass() * p0) / (4 * math.pi)) ** (1 / 3)
        t = dt * np.arange(1, nt + 1)
        y = P.forward(p0)
        ex = np.where(np.abs(r - t) < Reff, (r - t) / (2 * r), 0.0)
        cy, ce = np.cumsum(y, axis=0) * dt, np.cumsum(ex) * dt
        errs.append(np.abs(cy - ce[:, None]).max() / np.abs(ce).max())
        pos = (t > r - Reff) & (t < r)
        neg = (t > r) & (t < r + Reff)
        assert np.all(y[pos].mean(axis=0) > 0) and np.all(y[neg].mean(axis=0) < 0)
    assert errs[1] < 0.12 and errs[1] < 0.6 * errs[0]


# ---------------------------------------------------------------------------
# Prior factor, CGLS and RTO (Sec. 5 eqs. (extended-matrices), (normal-equations);
# Algorithm 1; App. A)
# ---------------------------------------------------------------------------

def _gext_dense(P, sigma, a):
    N = P.n_nodes
    G = P.forward(np.eye(N)).reshape(N, -1).T
    L = P.prior_apply(np.eye(N), a).T          # column i = L e_i
    return G, L, np.vstack([G / sigma, L])


def test_prior_factor_properties(tiny):
    P = tiny[0]
    N = P.n_nodes
    m = P.lumped_mass()
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(N), rng.standard_normal(N)
    for a in (0.0, 0.05):
        Lx = P.prior_apply(x, a)
        assert abs(Lx @ y - x @ P.prior_apply(y, a, transpose=True)) < 1e-13 * np.abs(Lx).max() * np.abs(y).sum()
        one = P.prior_apply(np.ones(N), a)               # K1 1 = 0  =>  L 1 = M_L^{1/2} 1
        np.testing.assert_allclose(one, np.sqrt(m), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(P.prior_apply(x, 0.0), np.sqrt(m) * x, rtol=1e-15)


def test_prior_factor_quadratic_on_kuhn_cube(cube8):
    """L = M_L^{-1/2}(M_L + a K1) at a != 0 in closed form (reading of the prior (I - a Delta_FE)^2,
    a -> 0 limit Sec. 4.1.1 eq. (iid-prior)).  On the Kuhn cube K1 is h times the 7-point stencil and
    M_L = h^3 at interior nodes, so for u = |x|^2 the stencil gives K1 u = -6 h^3 there and
    L u = h^{3/2} (u - 6 a): a wrong coefficient (a^2, 2a) or a dropped term moves every value.
    Likewise L^T (h^{3/2} u) = h^3 (u - 6 a) at nodes whose whole stencil is interior."""
    w, P = cube8
    n, h, a = 8, 1.0 / 8, 0.01
    idx = np.arange(n + 1)
    ii, jj, kk = np.meshgrid(idx, idx, idx, indexing="ij")
    node = (ii + (n + 1) * (jj + (n + 1) * kk)).ravel()
    xyz = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1) * h
    np.testing.assert_allclose(w.coords[node], xyz, atol=1e-15)   # lexicographic node numbering
    u = np.sum(w.coords ** 2, axis=1)
    inner = lambda lo, hi: node[((ii >= lo) & (ii <= hi) & (jj >= lo) & (jj <= hi) & (kk >= lo) & (kk <= hi)).ravel()]
    interior, deep = inner(1, n - 1), inner(2, n - 2)
    for aa in (a, 0.05):
        Lu = P.prior_apply(u, aa)
        np.testing.assert_allclose(Lu[interior], h ** 1.5 * (u[interior] - 6 * aa), rtol=1e-13, atol=1e-16)
        Ltu = P.prior_apply(h ** 1.5 * u, aa, transpose=True)
        np.testing.assert_allclose(Ltu[deep], h ** 3 * (u[deep] - 6 * aa), rtol=1e-13, atol=1e-17)
    # power of the check: the a-term is not small against the rounding bar
    assert np.abs(6 * a / u[interior]).min() > 1e-3


def test_prior_factor_uses_unit_coefficient_stiffness():
    """On a variable-speed ball, L (g . x) = M_L^{1/2} (g . x) at every interior node: the
    unit-coefficient stiffness annihilates linear functions there (sum over the support of
    vol_e grad(phi_i) is zero for an interior node), while the c^2-weighted K does not where c
    varies.  So a K-for-K1 swap fails here, which L 1 = M_L^{1/2} 1 cannot detect."""
    P, coords, tets, c = _tiny_ball(n=8, variable_c=True)
    m = P.lumped_mass()
    bnd = np.unique(_faces_numpy(tets))
    interior = np.setdiff1d(np.arange(P.n_nodes), bnd)
    g = np.array([0.3, -1.1, 0.7])
    u = coords @ g + 0.25
    for a in (0.01, 0.2):
        Lu = P.prior_apply(u, a)
        np.testing.assert_allclose(Lu[interior], np.sqrt(m[interior]) * u[interior], rtol=1e-12, atol=1e-14)
        # the alternative with K in place of K1 would miss by a clear margin
        Ku = P.matrix("K") @ u
        alt = (m * u + a * Ku) / np.sqrt(m)
        assert np.abs(alt[interior] - np.sqrt(m[interior]) * u[interior]).max() > 1e3 * 1e-12 * np.abs(Lu).max()
    assert np.ptp(c) > 0.05


def test_prior_factor_equals_assembled_matrices(tiny):
    """L x and L^T y equal (M_L x + a K1 x)/sqrt(M_L) and (M_L + a K1)(y/sqrt(M_L)) written with the
    assembled K1 (pinned by the stencil and identity tests) and the lumped masses."""
    P = tiny[0]
    N = P.n_nodes
    m = P.lumped_mass()
    K1 = P.matrix("K1")
    x = np.random.default_rng(9).standard_normal(N)
    for a in (0.01, 0.3):
        np.testing.assert_allclose(P.prior_apply(x, a), (m * x + a * (K1 @ x)) / np.sqrt(m), rtol=1e-12,
                                   atol=1e-14)
        t = x / np.sqrt(m)
        np.testing.assert_allclose(P.prior_apply(x, a, transpose=True), m * t + a * (K1 @ t), rtol=1e-12,
                                   atol=1e-14)


@pytest.mark.parametrize("reorth", [True, False])
def test_cgls_iterates_are_krylov_minimisers(tiny, reorth):
    P = tiny[0]
    sigma, a = 0.05, 0.02
    G, L, A = _gext_dense(P, sigma, a)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    bd = b[: G.shape[0]].reshape(1, P.n_steps, P.n_obs)
    bp = b[G.shape[0]:].reshape(1, -1)
    Atb = A.T @ b
    V = np.zeros((A.shape[1], 0))
    w = Atb.copy()
    for k in range(1, 7):
        # orthonormal basis of K_k(A^T A, A^T b), two Gram-Schmidt passes
        for _ in range(2):
            w -= V @ (V.T @ w)
        V = np.hstack([V, (w / np.linalg.norm(w))[:, None]])
        w = A.T @ (A @ V[:, -1])
        y, *_ = np.linalg.lstsq(A @ V, b, rcond=None)
        xk = V @ y
        x, res = P.cgls(bd, bp, sigma, a, k, reorth=reorth)
        assert np.linalg.norm(x[0] - xk) < 1e-9 * np.linalg.norm(xk)
        assert abs(res[0, -1] - np.linalg.norm(A @ x[0] - b)) < 1e-10 * np.linalg.norm(b)


def test_cgls_converges_to_least_squares(tiny):
    P = tiny[0]
    sigma, a = 0.05, 0.02
    G, L, A = _gext_dense(P, sigma, a)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((2, A.shape[0]))
    bd = b[:, : G.shape[0]].reshape(2, P.n_steps, P.n_obs)
    bp = b[:, G.shape[0]:]
    x, _ = P.cgls(bd, bp, sigma, a, 2 * P.n_nodes, reorth=True)
    for r in range(2):
        xs, *_ = np.linalg.lstsq(A, b[r], rcond=None)
        assert np.linalg.norm(x[r] - xs) < 1e-8 * np.linalg.norm(xs)


def test_float32_sweeps_round_like_float32(tiny):
    """The float32-state emulation of the sweeps (used only to measure the rounding floor of a
    float32 implementation) agrees with the float64 maps to the accumulated float32 rounding
    (between 1e-9 and 1e-5 relative over 20 steps), and keeps the transpose identity to that level."""
    P = tiny[0]
    rng = np.random.default_rng(13)
    p = rng.standard_normal((2, P.n_nodes))
    yh = rng.standard_normal((2, P.n_steps, P.n_obs))
    y, y32 = P.forward(p), P.forward_f32(p)
    a, a32 = P.adjoint(yh), P.adjoint_f32(yh)
    for ref, got in ((y, y32), (a, a32)):
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert 1e-9 < e < 1e-5
    lhs, rhs = np.sum(y32 * yh, axis=(1, 2)), np.sum(p * a32, axis=1)
    scale = np.linalg.norm(y32, axis=(1, 2)) * np.linalg.norm(yh, axis=(1, 2)) + \
        np.linalg.norm(p, axis=1) * np.linalg.norm(a32, axis=1)
    assert np.all(np.abs(lhs - rhs) < 1e-5 * scale)


def test_extended_residual_matches_least_squares(tiny):
    """The oracle's ||G_ext p - b|| of given samples (Sec. 5 eq. (lsqr-residual)) equals, at the
    least-squares solution, the residual numpy's lstsq reports, and at a fixed CGLS iterate the
    residual norm CGLS carries (itself pinned against the dense b - G_ext x above)."""
    P = tiny[0]
    sigma, a = 0.05, 0.02
    G, L, A = _gext_dense(P, sigma, a)
    N = P.n_nodes
    rng = np.random.default_rng(12)
    yobs = (G @ rng.standard_normal(N) + sigma * rng.standard_normal(G.shape[0])).reshape(P.n_steps, P.n_obs)
    S = 2
    eta = rng.standard_normal((S, P.n_steps, P.n_obs))
    xi = rng.standard_normal((S, N))
    for s in range(S):
        b = np.concatenate([yobs.ravel() / sigma + eta[s].ravel(), xi[s]])
        xs, rss, *_ = np.linalg.lstsq(A, b, rcond=None)
        got = P.extended_residual(xs[None], yobs, sigma, a, eta[s:s + 1], xi[s:s + 1])[0]
        assert abs(got - np.sqrt(rss[0])) < 1e-10 * np.linalg.norm(b)
    samples, res = P.rto(yobs, sigma, a, 7, eta, xi)
    got = P.extended_residual(samples, yobs, sigma, a, eta, xi)
    np.testing.assert_allclose(got, res[:, -1], rtol=1e-10)


@pytest.mark.parametrize("a", [0.02, 0.0])
def test_rto_sample_is_closed_form(tiny, a):
    """Converged RTO sample = C_post [G^T y / sigma^2 + G^T eta / sigma + Q p_prior] (App. A), with the
    prior precision Q = L^T L.  At a = 0 the prior is the paper's independent one, precision M_L
    (Sec. 4.1.1 eq. (iid-prior)), written here from the lumped masses alone, and p_prior = M_L^{-1/2} xi."""
    P = tiny[0]
    sigma = 0.05
    G, L, _ = _gext_dense(P, sigma, a)
    N = P.n_nodes
    if a == 0.0:
        m = P.lumped_mass()
        Q = np.diag(m)
        prior_mean = lambda x: x / np.sqrt(m)
    else:
        Q = L.T @ L
        prior_mean = lambda x: np.linalg.solve(L, x)
    rng = np.random.default_rng(6)
    yobs = G @ rng.standard_normal(N) + sigma * rng.standard_normal(G.shape[0])
    S = 3
    eta = rng.standard_normal((S, P.n_steps, P.n_obs))
    xi = rng.standard_normal((S, N))
    samples, _ = P.rto(yobs.reshape(P.n_steps, P.n_obs), sigma, a, 2 * N, eta, xi)
    Cpost = np.linalg.inv(G.T @ G / sigma ** 2 + Q)
    for s in range(S):
        ref = Cpost @ (G.T @ yobs / sigma ** 2 + G.T @ eta[s].ravel() / sigma + Q @ prior_mean(xi[s]))
        assert np.linalg.norm(samples[s] - ref) < 1e-8 * np.linalg.norm(ref)


def test_rto_distribution_matches_posterior():
    """Converged RTO samples have mean mu_post and covariance C_post (App. A), statistically."""
    P, *_ = _tiny_ball(n=3, n_steps=15, n_sens=6)
    sigma, a = 0.05, 0.02
    G, L, _ = _gext_dense(P, sigma, a)
    N = P.n_nodes
    rng = np.random.default_rng(7)
    yobs = G @ rng.standard_normal(N) + sigma * rng.standard_normal(G.shape[0])
    Cpost = np.linalg.inv(G.T @ G / sigma ** 2 + L.T @ L)
    mu = Cpost @ G.T @ yobs / sigma ** 2
    S = 3000
    eta = rng.standard_normal((S, P.n_steps, P.n_obs))
    xi = rng.standard_normal((S, N))
    samples, _ = P.rto(yobs.reshape(P.n_steps, P.n_obs), sigma, a, 2 * N, eta, xi)
    sd = np.sqrt(np.diag(Cpost))
    z = (samples.mean(axis=0) - mu) / (sd / math.sqrt(S))
    assert np.abs(z).max() < 4.5
    var_ratio = samples.var(axis=0, ddof=1) / sd ** 2
    assert np.abs(var_ratio - 1).max() < 5 * math.sqrt(2.0 / (S - 1))
    C = np.cov(samples.T)
    assert np.linalg.norm(C - Cpost) / np.linalg.norm(Cpost) < 6 / math.sqrt(S)


def test_posterior_std_follows_the_aperture():
    """Sec. 6.1 and 6.2: the pointwise posterior uncertainty falls as the measurement aperture grows and,
    for a partial aperture, grows with distance from it.  The first is exact for nested sensor sets at
    one noise level: each added sensor adds a positive semidefinite term to the posterior precision, so no
    diagonal entry of C_post can grow.  The second is a trend, checked by the rank correlation between
    a node's std and its distance to the nearest sensor over the nodes inside the sensor sphere."""
    from scipy.stats import spearmanr
    coords, post, _ = _dense.aperture_posteriors(oracle, W)
    sd = {k: v[0] for k, v in post.items()}
    assert np.all(sd["full"] <= sd["half"] * (1 + 1e-12))
    assert np.all(sd["half"] <= sd["quarter"] * (1 + 1e-12))
    assert sd["half"].mean() > 2 * sd["full"].mean() and sd["quarter"].mean() > 2 * sd["half"].mean()
    inside = np.linalg.norm(coords, axis=1) <= 0.7
    for name in ("half", "quarter"):
        std, pos = post[name]
        dist = _dense.distance_to_sensors(coords, pos)
        rho = spearmanr(dist[inside], std[inside]).correlation
        print(f"{name} aperture: rank correlation of std with distance to the sensors {rho:.3f}")
        assert rho > 0.6, (name, rho)


def test_stats_match_numpy():
    rng = np.random.default_rng(8)
    s = rng.standard_normal((7, 40)) * 3 + 1
    mean, std = oracle.stats(s)
    np.testing.assert_allclose(mean, s.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(std, s.std(axis=0, ddof=1), rtol=1e-13)


def test_noise_rule_gives_relative_level():
    """sigma from eq. (noise-model): ||sigma eta0|| / ||Y|| = d_noise exactly."""
    rng = np.random.default_rng(9)
    Y, e0 = rng.standard_normal((50, 12)), rng.standard_normal((50, 12))
    s = oracle.noise_sigma(Y, e0, 0.01, "l2")
    assert abs(np.linalg.norm(s * e0) / np.linalg.norm(Y) - 0.01) < 1e-15
    assert oracle.noise_sigma(Y, e0, 0.01, "max") == 0.01 * np.abs(Y).max()


def test_batched_rhs_equal_single_rhs(tiny):
    """Right-hand sides are independent: a batch of R gives bitwise the R single results."""
    P = tiny[0]
    rng = np.random.default_rng(10)
    p = rng.standard_normal((3, P.n_nodes))
    yh = rng.standard_normal((3, P.n_steps, P.n_obs))
    yb, pb = P.forward(p), P.adjoint(yh)
    xb, _ = P.cgls(yh, p, 0.1, 0.01, 7)
    for r in range(3):
        assert np.array_equal(yb[r], P.forward(p[r]))
        assert np.array_equal(pb[r], P.adjoint(yh[r]))
        x1, _ = P.cgls(yh[r:r + 1], p[r:r + 1], 0.1, 0.01, 7)
        assert np.array_equal(xb[r], x1[0])


@pytest.mark.parametrize("reorth", [True, False])
def test_lsqr_iterates_are_krylov_minimisers(tiny, reorth):
    """LSQR iterate k = the same Krylov-space minimiser as CGLS (Paige-Saunders LSQR)."""
    P = tiny[0]
    sigma, a = 0.05, 0.02
    G, L, A = _gext_dense(P, sigma, a)
    rng = np.random.default_rng(13)
    b = rng.standard_normal(A.shape[0])
    bd = b[: G.shape[0]].reshape(1, P.n_steps, P.n_obs)
    bp = b[G.shape[0]:].reshape(1, -1)
    V = np.zeros((A.shape[1], 0))
    w = A.T @ b
    for k in range(1, 7):
        for _ in range(2):
            w -= V @ (V.T @ w)
        V = np.hstack([V, (w / np.linalg.norm(w))[:, None]])
        w = A.T @ (A @ V[:, -1])
        y, *_ = np.linalg.lstsq(A @ V, b, rcond=None)
        xk = V @ y
        x, res, dg = P.lsqr(bd, bp, sigma, a, k, reorth=reorth, diag=True)
        assert np.linalg.norm(x[0] - xk) < 1e-9 * np.linalg.norm(xk)
        r = b - A @ x[0]
        nd = G.shape[0]
        assert abs(dg[0, -1, 0] - np.linalg.norm(r[:nd])) < 1e-10 * np.linalg.norm(b)
        assert abs(dg[0, -1, 1] - np.linalg.norm(r[nd:])) < 1e-10 * np.linalg.norm(b)
        assert abs(res[0, -1] - np.linalg.norm(r)) < 1e-10 * np.linalg.norm(b)


def test_lsqr_equals_cgls_and_converges(tiny):
    """With reorthogonalisation both solvers produce the same iterates; LSQR converges to lstsq."""
    P = tiny[0]
    sigma, a = 0.05, 0.02
    G, L, A = _gext_dense(P, sigma, a)
    rng = np.random.default_rng(14)
    b = rng.standard_normal((2, A.shape[0]))
    bd = b[:, : G.shape[0]].reshape(2, P.n_steps, P.n_obs)
    bp = b[:, G.shape[0]:]
    for k in (10, 60):
        xc, rc, dc = P.cgls(bd, bp, sigma, a, k, diag=True)
        xl, rl, dl = P.lsqr(bd, bp, sigma, a, k, diag=True)
        assert np.linalg.norm(xl - xc) < 1e-12 * np.linalg.norm(xc)
        np.testing.assert_allclose(dl, dc, rtol=1e-10, atol=1e-12)
    xl, _ = P.lsqr(bd, bp, sigma, a, 2 * P.n_nodes)
    for r in range(2):
        xs, *_ = np.linalg.lstsq(A, b[r], rcond=None)
        assert np.linalg.norm(xl[r] - xs) < 1e-8 * np.linalg.norm(xs)
    assert np.all(np.isfinite(xl))


# ---- counter-based perturbations (the sampler's own eta, xi) --------------------------------

def _numpy_philox_block(ctr, key):
    """numpy's Philox (4x64-10) advances its 256-bit counter before each block: start it at ctr - 1."""
    c = [int(x) for x in ctr]
    for i in range(4):                      # 256-bit decrement with borrow
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = (1 << 64) - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_matches_numpy():
    rng = np.random.default_rng(50)
    cases = [([1, 0, 0, 0], [0, 0]), ([0, 1, 0, 0], [0, 0]), ([0, 0, 0, 0], [1, 2]),
             ([2**64 - 1] * 4, [2**64 - 1] * 2)]
    cases += [(rng.integers(0, 2**64, 4, dtype=np.uint64, endpoint=False), rng.integers(0, 2**64, 2, dtype=np.uint64))
              for _ in range(200)]
    for ctr, key in cases:
        if all(int(x) == 0 for x in ctr):
            continue
        np.testing.assert_array_equal(oracle.philox4x64(ctr, key), _numpy_philox_block(ctr, key))


def test_normals_distribution():
    """Box-Muller on Philox words: every lane of the block is N(0, 1), pairs are independent."""
    from scipy import stats as st
    z = oracle.normals(123, 0, 0, 4, 2**20)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(st.skew(z.ravel())) < 5 * np.sqrt(6 / z.size)
    assert abs(st.kurtosis(z.ravel())) < 5 * np.sqrt(24 / z.size)
    for lane in range(4):                    # cos and sin branches of both pairs
        assert st.kstest(z[:, lane::4].ravel(), "norm").pvalue > 1e-4
    r2 = z[:, 0::2] ** 2 + z[:, 1::2] ** 2   # chi^2 with 2 degrees of freedom
    assert st.kstest(r2.ravel(), "expon", args=(0, 2)).pvalue > 1e-4
    # neighbouring lanes, streams, kinds and seeds are uncorrelated
    lim = 5 / np.sqrt(z.shape[1])
    for a, b in ((z[0, 0::4], z[0, 1::4]), (z[0, 0::4], z[0, 2::4]), (z[0], z[1])):
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(a.size)
    assert abs(np.corrcoef(z[0], oracle.normals(123, 1, 0, 1, 2**20)[0])[0, 1]) < lim
    assert abs(np.corrcoef(z[0], oracle.normals(124, 0, 0, 1, 2**20)[0])[0, 1]) < lim


def test_normals_stream_addressing():
    a = oracle.normals(7, 1, 0, 6, 37)
    np.testing.assert_array_equal(oracle.normals(7, 1, 3, 2, 37), a[3:5])
    np.testing.assert_array_equal(oracle.normals(7, 1, 0, 6, 10), a[:, :10])
    eta, xi = oracle.rto_normals(7, 6, 4, 9, 37)
    np.testing.assert_array_equal(xi, a)
    np.testing.assert_array_equal(eta.reshape(6, -1), oracle.normals(7, 0, 0, 6, 36))
