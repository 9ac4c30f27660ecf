"""Basis apply and its adjoint (oracle; test infrastructure only).

Each coil sensitivity is expanded on a basis, s_j = B c_j (Sec. II-B,
Eq. (5) and the Maxwell basis U_h of Sec. II-D).  B is either a dense
(N, K) matrix or Tucker-factored (Sec. II-E, Eqs. for the Tucker
decomposition and its truncated form):

    column k of B, reshaped C-order to (n0, n1, n2),
        = core[:, :, :, k] x_1 U0 x_2 U1 x_3 U2

with the k-mode product (A x_m U)[.., i, ..] = sum_p A[.., p, ..] U[i, p]
(Sec. II-E, the 1-mode product definition).  The factor shape is read as
U_m in C^{n_m x r_m}, which is what that mode-product definition needs (the
text prints the transposed shape for the truncated factors).  Factors are
shared by all K columns: a single 4-way Tucker with identity on mode 4.
"""
import numpy as np


def dense_apply(B: np.ndarray, c: np.ndarray) -> np.ndarray:
    """S[j] = B c_j ; B (N, K), c (J, K) -> S (J, N)."""
    B = np.asarray(B, dtype=np.complex128)
    c = np.asarray(c, dtype=np.complex128)
    return (B @ c.T).T


def dense_adjoint(B: np.ndarray, S: np.ndarray) -> np.ndarray:
    """c[j] = B^H S_j ; S (J, N) -> (J, K)."""
    B = np.asarray(B, dtype=np.complex128)
    S = np.asarray(S, dtype=np.complex128)
    return (B.conj().T @ S.T).T


def mode_product(A: np.ndarray, U: np.ndarray, mode: int) -> np.ndarray:
    """k-mode product: C[..., i, ...] = sum_p A[..., p, ...] U[i, p] along axis ``mode``."""
    A = np.moveaxis(np.asarray(A), mode, 0)
    shp = A.shape
    C = np.asarray(U) @ A.reshape(shp[0], -1)
    return np.moveaxis(C.reshape((U.shape[0],) + shp[1:]), 0, mode)


def tucker_coil_map(U, core: np.ndarray, cj: np.ndarray) -> np.ndarray:
    """One coil map s_j = B c_j as an (n0, n1, n2) array.

    The basis index is contracted first (core x_4 c_j), then the three
    spatial mode products, as the Tucker form of the basis states.
    """
    core = np.asarray(core, dtype=np.complex128)
    T = core.reshape(-1, core.shape[-1]) @ np.asarray(cj, dtype=np.complex128)
    T = T.reshape(core.shape[:-1])
    for m in range(3):
        T = mode_product(T, np.asarray(U[m], dtype=np.complex128), m)
    return T


def tucker_apply(U, core: np.ndarray, c: np.ndarray) -> np.ndarray:
    """S (J, N) for a Tucker-factored basis, one coil at a time."""
    c = np.asarray(c, dtype=np.complex128)
    return np.stack([tucker_coil_map(U, core, c[j]).reshape(-1) for j in range(c.shape[0])])


def tucker_adjoint(U, core: np.ndarray, S: np.ndarray) -> np.ndarray:
    """c[j] = B^H S_j for a Tucker-factored basis.

    B^H applies the adjoint of each step in reverse order: the mode products
    with U_m^H, then the contraction with the conjugated core.
    """
    core = np.asarray(core, dtype=np.complex128)
    dims = tuple(u.shape[0] for u in U)
    S = np.asarray(S, dtype=np.complex128)
    out = []
    for j in range(S.shape[0]):
        T = S[j].reshape(dims)
        for m in (2, 1, 0):
            T = mode_product(T, np.asarray(U[m], dtype=np.complex128).conj().T, m)
        out.append(core.reshape(-1, core.shape[-1]).conj().T @ T.reshape(-1))
    return np.stack(out)


def tucker_materialise(U, core: np.ndarray) -> np.ndarray:
    """Dense (N, K) matrix of a Tucker basis (only for small shapes)."""
    core = np.asarray(core, dtype=np.complex128)
    K = core.shape[-1]
    cols = []
    for k in range(K):
        T = core[..., k]
        for m in range(3):
            T = mode_product(T, np.asarray(U[m], dtype=np.complex128), m)
        cols.append(T.reshape(-1))
    return np.stack(cols, axis=1)
