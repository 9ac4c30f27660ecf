"""Pins for the oracle's accuracy-controlled Tucker compression (ST-HOSVD).

* A basis that is exactly Tucker of ranks r is recovered with those ranks and reconstructed to
  rounding, at a tiny eps.
* For random bases and several eps the reconstruction error obeys ||B - B~|| <= eps ||B||, and
  its square equals the sum of the discarded squared singular values (the ST-HOSVD identity).
* eps = 0 keeps every rank (up to the unfolding's row count) and reconstructs exactly.
* The factors have orthonormal columns; the core's norm equals the kept energy.
"""
import numpy as np
import pytest

from oracle.basis import tucker_materialise
from oracle.compress import reconstruct, st_hosvd
from synth import complex_normal, rng_for, tucker_basis


def test_exact_tucker_is_recovered():
    dims, ranks, K = (8, 10, 6), (3, 4, 2), 5
    U, core = tucker_basis(rng_for(41, 2), dims, ranks, K, 3, 1.5)
    B = tucker_materialise(U, core)
    Us, G, r, dropped = st_hosvd(B, dims, 1e-10)
    assert r == list(ranks)
    assert np.linalg.norm(reconstruct(Us, G) - B) < 1e-12 * np.linalg.norm(B)


@pytest.mark.parametrize("eps", [0.3, 0.1, 0.01])
def test_error_bound_and_identity(eps):
    rng = np.random.default_rng(42)
    dims, K = (8, 7, 6), 4
    # a tensor with a decaying spectrum in every mode
    B = complex_normal(rng, (int(np.prod(dims)), K))
    for m, n in enumerate(dims):
        w = np.exp(-0.6 * np.arange(n))
        shape = [1, 1, 1, 1]
        shape[m] = n
        B = (B.reshape(*dims, K) * w.reshape(shape)).reshape(-1, K)
    Us, G, r, dropped = st_hosvd(B, dims, eps)
    err2 = np.linalg.norm(reconstruct(Us, G) - B) ** 2
    total = np.linalg.norm(B) ** 2
    assert err2 <= eps * eps * total * (1 + 1e-12)
    assert abs(err2 - sum(dropped)) <= 1e-10 * total
    for u in Us:
        assert np.max(np.abs(u.conj().T @ u - np.eye(u.shape[1]))) < 1e-12
    assert abs(np.linalg.norm(G) ** 2 - (total - err2)) <= 1e-10 * total
    if eps >= 0.1:
        assert any(ri < n for ri, n in zip(r, dims))


def test_eps_zero_keeps_everything():
    rng = np.random.default_rng(43)
    dims, K = (5, 4, 3), 2
    B = complex_normal(rng, (int(np.prod(dims)), K))
    Us, G, r, _ = st_hosvd(B, dims, 0.0)
    assert r == [5, 4, 3]
    assert np.linalg.norm(reconstruct(Us, G) - B) < 1e-12 * np.linalg.norm(B)
