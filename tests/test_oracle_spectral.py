"""Pins of the spectral-prior oracle (oracle/spectral.py) against closed forms.

* Covariance: the exact discrete covariance function of the grid field,
  ifftn(a^2), has value sigma^2 at lag 0 and follows the Matern closed forms
  sigma^2 (1 + r/ell) e^{-r/ell} (expo = nu + d/2 = 3, nu = 3/2, the paper's
  setting) and sigma^2 (1 + r/ell + r^2/(3 ell^2)) e^{-r/ell} (expo = 4, nu = 5/2)
  along an axis, on a grid fine and large against ell.
* The filter applied twice to an impulse gives that covariance column.
* Trilinear interpolation reproduces trilinear functions; rows sum to one.
* P and P^T are transposes.
* Latent RTO: iterate k is the Krylov-space least-squares minimiser, and the
  converged iterate is the dense least-squares solution of
  [G P / sigma ; I] w = [y/sigma + eta ; xi].
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.spectral import SpectralPrior, latent_residual, latent_rto


@pytest.mark.parametrize("expo,shape", [(3.0, lambda x: (1 + x) * np.exp(-x)),
                                        (4.0, lambda x: (1 + x + x * x / 3) * np.exp(-x))])
def test_covariance_is_matern(expo, shape):
    pr = SpectralPrior(n=128, lo=-2.0, side=4.0, ell=0.25, sigma=3.0, expo=expo)
    cov = np.fft.ifftn(pr.amplitude() ** 2).real
    assert cov[0, 0, 0] == pytest.approx(9.0, rel=1e-12)
    m = np.arange(0, 40)
    r = m * pr.h
    ref = 9.0 * shape(r / pr.ell)
    for line in (cov[0, 0, m], cov[0, m, 0], cov[m, 0, 0]):
        assert np.max(np.abs(line - ref)) < 2e-3 * 9.0


def test_filter_twice_gives_covariance():
    pr = SpectralPrior(n=16, lo=-1.25, side=2.5, ell=0.3, sigma=2.0)
    e0 = np.zeros(pr.size)
    e0[0] = 1.0
    col = pr.field(pr.field(e0)).reshape(16, 16, 16)
    np.testing.assert_allclose(col, np.fft.ifftn(pr.amplitude() ** 2).real, rtol=0, atol=1e-12)


def test_interpolation_exact_for_trilinear():
    pr = SpectralPrior(n=12, lo=-1.25, side=2.5, ell=0.3, sigma=1.0)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1.2, 1.0, size=(500, 3))

    def f(x, y, z):
        return 1 + 2 * x - y + 0.5 * z + 0.3 * x * y * z - 0.7 * y * z

    g = pr.lo + pr.h * np.arange(pr.n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    I = pr.interp_matrix(pts)
    np.testing.assert_allclose(I @ f(X, Y, Z).ravel(), f(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.asarray(I.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-14)


def _tiny():
    coords, tets = W.ball_mesh(3)
    w = W.Workload(name="tiny", coords=coords, tets=tets, c_tet=None, absorbing=True, dt=0.2 * 2 / 3, n_steps=15,
                   sensor_pos=W.fibonacci_sphere(6, 0.7), p0_true=W.smooth_bump(coords, 0.8))
    return w, oracle.Problem.from_workload(w)


def test_transpose_pair():
    w, O = _tiny()
    pr = SpectralPrior(n=8, lo=-1.25, side=2.5, ell=0.3, sigma=3.0)
    I = pr.interp_matrix(w.coords)
    rng = np.random.default_rng(6)
    a = rng.standard_normal((2, pr.size))
    v = rng.standard_normal((2, w.n_nodes))
    lhs = np.sum(pr.apply(a, I) * v, axis=1)
    rhs = np.sum(a * pr.apply_t(v, I), axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_latent_rto_krylov_and_converged():
    w, O = _tiny()
    pr = SpectralPrior(n=6, lo=-1.25, side=2.5, ell=0.4, sigma=3.0)
    I = pr.interp_matrix(w.coords)
    n = pr.size
    sigma = 0.05
    P = pr.apply(np.eye(n), I).T                       # N x n
    G = O.forward(np.eye(w.n_nodes)).reshape(w.n_nodes, -1).T
    A = np.vstack([G @ P / sigma, np.eye(n)])
    rng = np.random.default_rng(7)
    yobs = rng.standard_normal((w.n_steps, w.n_obs)) * 0.1
    eta = rng.standard_normal((2, w.n_steps, w.n_obs))
    xi = rng.standard_normal((2, n))
    b = [np.concatenate([(yobs / sigma + eta[r]).ravel(), xi[r]]) for r in range(2)]
    # Krylov minimiser after k iterations
    for k in (1, 3, 6):
        p0, lat, res = latent_rto(O, pr, I, yobs, sigma, k, eta, xi)
        for r in range(2):
            # orthonormal basis of span{A^T b, (A^T A) A^T b, ...} by Arnoldi with reorthogonalisation
            Qk = np.zeros((n, 0))
            v = A.T @ b[r]
            for _ in range(k):
                for _ in range(2):
                    v = v - Qk @ (Qk.T @ v)
                Qk = np.hstack([Qk, (v / np.linalg.norm(v))[:, None]])
                v = A.T @ (A @ Qk[:, -1])
            y, *_ = np.linalg.lstsq(A @ Qk, b[r], rcond=None)
            ref = Qk @ y
            assert np.linalg.norm(lat[r] - ref) < 1e-8 * np.linalg.norm(ref)
            assert abs(res[r, -1] - np.linalg.norm(b[r] - A @ lat[r])) < 1e-10 * np.linalg.norm(b[r])
    # the recomputed residual of given latent samples equals the dense one
    p0, lat, res = latent_rto(O, pr, I, yobs, sigma, 4, eta, xi)
    got = latent_residual(O, pr, I, lat, yobs, sigma, eta, xi)
    for r in range(2):
        assert abs(got[r] - np.linalg.norm(b[r] - A @ lat[r])) < 1e-12 * np.linalg.norm(b[r])
    # converged
    p0, lat, res = latent_rto(O, pr, I, yobs, sigma, n, eta, xi)
    for r in range(2):
        ref, rss, *_ = np.linalg.lstsq(A, b[r], rcond=None)
        assert np.linalg.norm(lat[r] - ref) < 1e-9 * np.linalg.norm(ref)
        assert abs(latent_residual(O, pr, I, ref, yobs, sigma, eta[r], xi[r])[0] - np.sqrt(rss[0])) \
            < 1e-10 * np.linalg.norm(b[r])
        np.testing.assert_allclose(p0[r], P @ lat[r], rtol=0, atol=1e-10 * np.abs(p0[r]).max())


def test_float32_floor_of_the_latent_std():
    """The rounding floor behind the float32 latent-RTO test: on ball16 (16^3 grid, ell = 0.2,
    64 samples) float32 sweeps in the velocity form (oracle/float32_floor.py, numpy float32) give a
    posterior std 1.0e-4 away from the float64 oracle after 20 iterations while samples and mean
    stay near 4e-6; the one-vector (three-level) form that the GPU sweeps use gives 4e-5 there, and
    the oracle's float32 literal three-substep sweeps 4e-5."""
    from oracle.float32_floor import StaggeredFloat32, ThreeLevel
    w = W.make_workload("ball16")
    O = oracle.Problem.from_workload(w)
    pr = SpectralPrior(16, -1.25, 2.5, 0.2, 3.0)
    I = pr.interp_matrix(w.coords)
    Y, yobs, sigma = oracle.synthesize(O, w)
    S, n_iter = 64, 20
    rng = np.random.default_rng(41)
    eta = rng.standard_normal((S, w.n_steps, w.n_obs))
    xi = rng.standard_normal((S, pr.size))
    ref, _, _ = latent_rto(O, pr, I, yobs, sigma, n_iter, eta, xi)
    m0, s0 = oracle.stats(ref)
    rl = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    stag, _, _ = latent_rto(StaggeredFloat32(O), pr, I, yobs, sigma, n_iter, eta, xi)
    three, _, _ = latent_rto(ThreeLevel(O), pr, I, yobs, sigma, n_iter, eta, xi)
    lit, _, _ = latent_rto(O, pr, I, yobs, sigma, n_iter, eta, xi, sweeps="f32")
    (ms, ss), (m3, s3), (ml, sl) = oracle.stats(stag), oracle.stats(three), oracle.stats(lit)
    assert rl(stag, ref) < 1e-5 and rl(ms, m0) < 1e-5
    assert 7e-5 < rl(ss, s0) < 1.5e-4
    assert rl(three, ref) < 1e-5 and rl(m3, m0) < 1e-5 and rl(s3, s0) < 7e-5
    assert rl(sl, s0) < 7e-5
