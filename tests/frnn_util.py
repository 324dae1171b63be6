"""Helpers shared by the tests of the grid-transformation network: random
rotations, block voxel centres, and a network built by hand to represent
R^T P exactly (pairs of ReLU units carry each rotation entry as
relu(x) - relu(-x)).  Input generation only."""
import numpy as np

H = 32


def random_rotations(n, seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def centres(m):
    w = 2 * m
    jz, jy, jx = np.meshgrid(np.arange(w), np.arange(w), np.arange(w), indexing="ij")
    return np.stack([(jx + 0.5) / m - 1, (jy + 0.5) / m - 1, (jz + 0.5) / m - 1], -1).reshape(-1, 3)


def exact_params(m):
    P = centres(m)
    V = P.shape[0]
    W1 = np.zeros((H, 9))
    for k in range(9):
        W1[2 * k, k] = 1.0
        W1[2 * k + 1, k] = -1.0
    b1 = np.zeros(H)
    W2 = np.zeros((3 * V, H))
    for j in range(V):
        for a in range(3):
            for b in range(3):
                k = 3 * b + a                      # x_k = R[b][a]
                W2[3 * j + a, 2 * k] = P[j, b]
                W2[3 * j + a, 2 * k + 1] = -P[j, b]
    return np.concatenate([W1.ravel(), b1, W2.ravel(), np.zeros(3 * V)])
