"""The library's host pole extraction (chi0_lanczos_poles) against its definition.

The poles of alpha_k are the eigenvalues of the tridiagonal T_k and the
residues |c|^2 times the squared first components of its normalised
eigenvectors.  Checked against a dense eigen-decomposition (LAPACK through
NumPy) of random tridiagonals and of the oracle's Lanczos tridiagonal of a
molecule, and through the pole sum, which must reproduce the oracle's
alpha_k(w) from a dense solve with T_k.  No GPU: the routine runs on the host.
"""
import numpy as np
import pytest

from oracle import lanczos_oracle as lo
from paper_1005_5340_amd import chi0, synth


def _dense(a, b):
    k = len(a)
    return np.diag(a) + np.diag(b[: k - 1], 1) + np.diag(b[: k - 1], -1)


@pytest.mark.parametrize("k", [1, 2, 3, 17, 300])
def test_random_tridiagonal(k):
    rng = np.random.default_rng(k)
    a = rng.standard_normal(k) * 3
    b = np.abs(rng.standard_normal(k))
    th, r = chi0.lanczos_poles(a, b, 1.7)
    w, U = np.linalg.eigh(_dense(a, b))
    scale = np.abs(w).max()
    assert np.all(np.diff(th) >= 0)
    assert np.abs(th - w).max() <= 1e-13 * scale
    assert np.abs(r - 1.7 * U[0] ** 2).max() <= 1e-12
    assert abs(r.sum() - 1.7) <= 1e-12


def test_split_and_clustered():
    # zero off-diagonals split the matrix: only the block holding e_1 carries weight
    a = np.array([1.0, 1.0, 1.0, 2.0, 2.0])
    b = np.array([0.0, 1e-20, 0.0, 0.0, 0.0])
    th, r = chi0.lanczos_poles(a, b, 1.0)
    np.testing.assert_allclose(th, [1, 1, 1, 2, 2], rtol=1e-15)
    np.testing.assert_allclose(r, [1, 0, 0, 0, 0], atol=1e-15)
    # tight cluster around 1 (eigenvalues 1 + 2e-8 cos(j pi / 51))
    th, r = chi0.lanczos_poles(np.ones(50), np.full(49, 1e-8), 1.0)
    exact = 1 + 2e-8 * np.cos(np.arange(1, 51) * np.pi / 51)
    np.testing.assert_allclose(th, np.sort(exact), rtol=0, atol=4e-15)   # a few ulps of 1
    assert abs(r.sum() - 1.0) <= 1e-14


def test_molecule_tridiagonal_pole_sum():
    sys = synth.make_system("atoms4_orb4", seed=0)
    d = sys.drives("z")[0]
    Om2 = lo.casida_matrix(sys)
    a, b, cn2 = lo.lanczos(Om2, lo.start_vector(sys, d), 40)
    th, r = chi0.lanczos_poles(a, b, cn2)
    tho, ro = lo.poles(a, b, cn2)
    assert np.abs(th - tho).max() <= 1e-12 * np.abs(tho).max()
    assert np.abs(r - ro).max() <= 1e-12 * cn2
    om = np.linspace(0.0, 1.5, 31)
    z = (om + 1j * sys.eps) ** 2
    pole_sum = (r[None, :] / (th[None, :] - z[:, None])).sum(1)
    ref = lo.spectrum(a, b, cn2, om, sys.eps)
    assert np.abs(pole_sum - ref).max() <= 1e-9 * np.abs(ref).max()


def test_errors():
    with pytest.raises(chi0.Chi0Error):
        chi0.lanczos_poles(np.array([1.0, np.nan]), np.array([1.0]), 1.0)
    with pytest.raises(chi0.Chi0Error):
        chi0.lanczos_poles(np.array([1.0]), np.array([0.0]), -1.0)
    L = chi0.lib()
    assert L.chi0_lanczos_poles(0, None, None, 1.0, None, None) == -1
