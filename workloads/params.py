"""Seeded random draws that the method takes as inputs (numpy PCG64, float32).

  * initial weights and biases, each drawn from U(-1/sqrt(fan_in), +1/sqrt(fan_in))
    in the canonical flat layout W1, b1, W2, b2, ... with W_l row-major [out][in];
  * the Fourier feature matrix B (m x 3) with entries N(0, sigma^2);
  * the positional-encoding matrix (rows 2^(k-1) e_d), which involves no draw;
  * the permutation that defines one epoch.
"""
import numpy as np


def net_shapes(K, W, H, c):
    return [(W, K)] + [(W, W)] * (H - 1) + [(c, W)]


def init_params(K, W, H, c, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for (n_out, n_in) in net_shapes(K, W, H, c):
        a = 1.0 / np.sqrt(n_in)
        parts.append(rng.uniform(-a, a, size=n_out * n_in))
        parts.append(rng.uniform(-a, a, size=n_out))
    return np.concatenate(parts).astype(np.float32)


def ffm_matrix(m, sigma, seed):
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal((m, 3))).astype(np.float32)


def pe_matrix(L):
    B = np.zeros((3 * L, 3), dtype=np.float32)
    for k in range(L):
        for d in range(3):
            B[3 * k + d, d] = 2.0 ** (k - 1)
    return B


def epoch_permutation(n, seed):
    return np.random.default_rng(seed).permutation(n).astype(np.int64)
