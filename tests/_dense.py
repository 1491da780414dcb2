"""Dense-matrix helpers for pinning the oracle on tiny meshes.

These build the paper's operators as explicit matrices from the assembled
K, B, M_L that the oracle exports, using the paper's *block-matrix* and
*factored* forms (Sec. 3 eq. (matrix-stromer), App. B), which are different
formulas from the substep form the oracle time-steps with.
"""
import numpy as np


def propagator_block(K, B, m, dt):
    """A_dt from its 2x2 block form, eq. (matrix-stromer)."""
    N = K.shape[0]
    I = np.eye(N)
    Mi = np.diag(1.0 / m)
    MK, MB = Mi @ K, Mi @ B
    top = np.hstack([I - dt ** 2 / 2 * MK, dt * I - dt ** 2 / 2 * MB - dt ** 3 / 4 * MK])
    bot = np.hstack([-dt * MK, I - dt * MB - dt ** 2 / 2 * MK])
    return np.vstack([top, bot])


def propagator_factors(K, B, m, dt):
    """S1, S2, S3, S4 of App. B, with A_dt = S4 S3 S2 S1."""
    N = K.shape[0]
    I, Z = np.eye(N), np.zeros((N, N))
    S1 = np.block([[I, dt / 2 * I], [Z, I]])
    S2 = np.block([[I, Z], [-dt * K, np.diag(m) - dt * B]])
    S3 = np.block([[I, Z], [Z, np.diag(1.0 / m)]])
    S4 = S1.copy()
    return S1, S2, S3, S4


def sensor_matrix(nodes, weights, N):
    """Pi restricted to the pressure block: [N_obs][N]."""
    Pi = np.zeros((nodes.shape[0], N))
    for s in range(nodes.shape[0]):
        for k in range(4):
            Pi[s, nodes[s, k]] += weights[s, k]
    return Pi


def forward_matrix(A, Pi, n_steps):
    """G of eq. (discrete-wave-matrix) acting on p0 (z0 = (p0, 0)): rows (n, s), n = 1..N_T."""
    N = Pi.shape[1]
    rows = []
    An = np.eye(2 * N)
    for _ in range(n_steps):
        An = A @ An
        rows.append(Pi @ An[:N, :N])
    return np.vstack(rows)


def aperture_posteriors(oracle, W, n=6, n_steps=40, n_sens=160):
    """Exact pointwise posterior std for three nested measurement apertures.

    A ball of n cells per axis (absorbing, c = 1, dt = 0.2 h) with sensors on the
    sphere r = 0.7: all of them, the half z > 0, and the quarter z > 0, x > 0.  The
    prior precision is M_L (the paper's independent prior, eq. (iid-prior)); one
    noise level sigma = 0.01 max|G_full| serves all three.  Returns the node
    coordinates, {name: (std, sensor positions)} and sigma.
    """
    coords, tets = W.ball_mesh(n)
    allpos = W.fibonacci_sphere(n_sens, 0.7)
    sets = {"full": allpos, "half": allpos[allpos[:, 2] > 0],
            "quarter": allpos[(allpos[:, 2] > 0) & (allpos[:, 0] > 0)]}
    out, sigma = {}, None
    for name, pos in sets.items():
        P = oracle.Problem(coords, tets, None, True, 0.2 * 2.0 / n, n_steps, sensor_pos=pos)
        N = P.n_nodes
        G = P.forward(np.eye(N)).reshape(N, -1).T
        if sigma is None:
            sigma = 0.01 * float(np.abs(G).max())
        H = G.T @ G / sigma ** 2 + np.diag(P.lumped_mass())
        out[name] = (np.sqrt(np.diag(np.linalg.inv(H))), pos)
    return coords, out, sigma


def distance_to_sensors(coords, pos):
    """Distance of each node to its nearest sensor."""
    return np.min(np.linalg.norm(coords[:, None, :] - pos[None, :, :], axis=2), axis=1)
