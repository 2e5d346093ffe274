"""Pins of the GMRES error-estimate oracle (stopping test of Sec. 4.1).

The oracle computes, at every Krylov dimension k, the GMRES iterate from a
dense least-squares solve and the estimates eps_X = |pinv(H_k)|_F |r| / |x|
and eps_P = |pinv(H_k)|_F |d.r| / |d.x|.  These tests tie it to facts
that do not come from its own code:

* at full dimension the Hessenberg matrix is unitarily similar to A, so the
  Frobenius norm of its inverse equals |A^-1|_F (closed form for a diagonal
  A, a dense inverse for a general one), and the iterate is A^-1 b;
* the GMRES iterate of dimension k minimises |b - A x| over x0 + K_k, checked
  against a least-squares fit over an orthonormalised explicit Krylov matrix
  [r0, A r0, ..., A^{k-1} r0];
* the residual never grows with k, and both estimates vanish as x -> A^-1 b;
* a start x0 != 0 gives the same iterates as solving for the correction.

Planted mistakes (the norm of H_k instead of its pseudo-inverse, a conjugated
d in P, a dropped start vector) each fail one of the pins.
"""
import numpy as np
import pytest

from oracle import gmres_oracle as go


def _rand_system(n, seed, cond=1.0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * (1.0 + cond) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    d = rng.standard_normal(n) + 0.5j * rng.standard_normal(n)
    return A, b, d


def test_full_dimension_diagonal_closed_form():
    lam = np.array([0.5, -1.0 + 0.2j, 2.0, 3.0j, -0.25, 1.5 - 0.5j])
    A = np.diag(lam)
    b = np.ones(lam.size, complex)
    d = np.arange(1.0, lam.size + 1.0)
    tr = go.gmres_eps_trace(A, b, d, kmax=lam.size)
    assert tr["k"][-1] == lam.size
    np.testing.assert_allclose(tr["ainv_f"][-1], np.sqrt(np.sum(1.0 / np.abs(lam) ** 2)), rtol=1e-12)
    np.testing.assert_allclose(tr["x"], b / lam, rtol=1e-12)
    np.testing.assert_allclose(tr["p"][-1], d @ (b / lam), rtol=1e-12)
    assert tr["eps_x"][-1] < 1e-13 and tr["eps_p"][-1] < 1e-13


def test_full_dimension_general_matrix():
    A, b, d = _rand_system(12, 1)
    tr = go.gmres_eps_trace(A, b, d, kmax=12)
    np.testing.assert_allclose(tr["ainv_f"][-1], np.linalg.norm(np.linalg.inv(A), "fro"), rtol=1e-10)
    np.testing.assert_allclose(tr["x"], np.linalg.solve(A, b), rtol=1e-10)
    np.testing.assert_allclose(tr["p"][-1], d @ np.linalg.solve(A, b), rtol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_iterate_minimises_residual_over_explicit_krylov_space(k):
    A, b, d = _rand_system(20, 2)
    rng = np.random.default_rng(9)
    x0 = 0.1 * (rng.standard_normal(20) + 1j * rng.standard_normal(20))
    tr = go.gmres_eps_trace(A, b, d, kmax=k, x0=x0)
    r0 = b - A @ x0
    Kr = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], axis=1)
    Q, _ = np.linalg.qr(Kr)
    c = np.linalg.lstsq(A @ Q, r0, rcond=None)[0]
    best = np.linalg.norm(r0 - A @ Q @ c) / np.linalg.norm(r0)
    np.testing.assert_allclose(tr["res"][k - 1], best, rtol=1e-9)
    np.testing.assert_allclose(tr["x"], x0 + Q @ c, rtol=1e-8, atol=1e-12)


def test_residual_monotone_and_estimates_vanish():
    A, b, d = _rand_system(30, 3, cond=0.5)
    tr = go.gmres_eps_trace(A, b, d, kmax=30)
    assert np.all(np.diff(tr["res"]) <= 1e-12)
    assert tr["eps_x"][-1] < 1e-10 and tr["eps_p"][-1] < 1e-10
    assert tr["eps_x"][0] > 1e-3


def test_start_vector_is_a_correction():
    A, b, d = _rand_system(16, 4)
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    t1 = go.gmres_eps_trace(A, b, d, kmax=6, x0=x0)
    t2 = go.gmres_eps_trace(A, b - A @ x0, d, kmax=6)
    np.testing.assert_allclose(t1["x"], x0 + t2["x"], rtol=1e-10)
    np.testing.assert_allclose(t1["res"], t2["res"], rtol=1e-10)


# --------------------------------------------------------- planted mistakes
def _pins_pass():
    try:
        test_full_dimension_diagonal_closed_form()
        test_full_dimension_general_matrix()
        for k in (1, 2, 4, 7):
            test_iterate_minimises_residual_over_explicit_krylov_space(k)
        test_start_vector_is_a_correction()
    except AssertionError:
        return False
    return True


def test_mutation_norm_instead_of_inverse(monkeypatch):
    real_pinv = np.linalg.pinv

    class FakeLinalg:
        def __getattr__(self, name):
            if name == "pinv":
                return lambda M, *a, **k: M.conj().T     # |H_k|_F, not |pinv(H_k)|_F
            return getattr(np.linalg, name)

    class FakeNp:
        def __getattr__(self, name):
            return FakeLinalg() if name == "linalg" else getattr(np, name)

    monkeypatch.setattr(go, "np", FakeNp())
    assert not _pins_pass()
    monkeypatch.undo()
    assert np.linalg.pinv is real_pinv and _pins_pass()


def test_mutation_conjugated_drive(monkeypatch):
    orig = go.gmres_eps_trace

    def conj_d(A, b, d, kmax, x0=None):
        return orig(A, b, np.conj(np.asarray(d, complex)), kmax, x0)

    monkeypatch.setattr(go, "gmres_eps_trace", conj_d)
    assert not _pins_pass()


def test_mutation_dropped_start(monkeypatch):
    orig = go.gmres_eps_trace

    def no_x0(A, b, d, kmax, x0=None):
        return orig(A, b, d, kmax, None)

    monkeypatch.setattr(go, "gmres_eps_trace", no_x0)
    assert not _pins_pass()
