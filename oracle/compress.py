"""Accuracy-controlled Tucker compression of a dense basis (oracle; test infrastructure only).

Paper, Sec. II-E, Eqs. (truncated_tucker) and (tucker_error): the basis, reshaped column by
column onto the image grid, is approximated by a truncated Tucker expansion with
||T - G x1 U1 x2 U2 x3 U3|| < eps ||T||.  Here T is the 4-way tensor n0 x n1 x n2 x K (the
columns along mode 4, which is kept whole: factors shared by all columns, as in the rest of
this code), and the expansion is computed by the sequentially truncated higher-order SVD
(Vannieuwenhoven, Vandebril and Meerbergen, SIAM J. Sci. Comput. 34, 2012): for modes
m = 1, 2, 3 in turn, the left singular vectors of the mode-m unfolding of the current,
already truncated tensor, keeping the fewest r_m whose discarded squared singular values sum
to at most eps^2 ||T||^2 / 3, then projecting that mode onto them.  The squared error is the
sum of the discarded squared singular values, so ||T - T~|| <= eps ||T||.
"""
import numpy as np

from .basis import mode_product


def unfold(Y: np.ndarray, m: int) -> np.ndarray:
    """Mode-m unfolding: rows indexed by axis m, columns by the other axes in C order."""
    return np.moveaxis(Y, m, 0).reshape(Y.shape[m], -1)


def st_hosvd(B: np.ndarray, dims, eps: float):
    """B (N, K) with N = prod(dims) -> (U [3 x (n_m, r_m)], core (r0, r1, r2, K), ranks,
    discarded squared norm per mode)."""
    K = B.shape[1]
    T = np.asarray(B, dtype=np.complex128).T.reshape((K,) + tuple(dims))  # (K, n0, n1, n2)
    Y = np.moveaxis(T, 0, -1)                                               # (n0, n1, n2, K)
    total = float(np.linalg.norm(Y) ** 2)
    budget = eps * eps * total / 3.0
    Us, ranks, dropped = [], [], []
    for m in range(3):
        Um, s, _ = np.linalg.svd(unfold(Y, m), full_matrices=False)
        s2 = s ** 2
        tail = np.concatenate([np.cumsum(s2[::-1])[::-1], [0.0]])  # tail[r] = sum_{i >= r} s_i^2
        r = int(np.argmax(tail <= budget))
        r = max(r, 1)
        Us.append(Um[:, :r])
        ranks.append(r)
        dropped.append(float(tail[r]))
        Y = mode_product(Y, Um[:, :r].conj().T, m)
    return Us, Y, ranks, dropped


def reconstruct(Us, core) -> np.ndarray:
    """G x1 U1 x2 U2 x3 U3 -> (N, K)."""
    Y = core
    for m in range(3):
        Y = mode_product(Y, Us[m], m)
    K = Y.shape[-1]
    return Y.reshape(-1, K)
