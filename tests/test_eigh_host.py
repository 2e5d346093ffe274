"""The library's host Jacobi eigen-solver (used for the warm-start basis)."""
import numpy as np
import pytest

from paper_1005_5340_amd import chi0


@pytest.mark.parametrize("n", [1, 3, 17, 64])
def test_jacobi_matches_definition(n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = B @ B.conj().T
    w, V = chi0.debug_eigh(A)
    assert np.all(np.diff(w) <= 1e-12 * w.max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(V @ np.diag(w) @ V.conj().T - A).max() < 1e-12 * np.abs(A).max()
    assert np.abs(w - np.sort(np.linalg.eigvalsh(A))[::-1]).max() < 1e-12 * w.max()
