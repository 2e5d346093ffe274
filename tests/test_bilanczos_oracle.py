"""Pins of the two-sided (biorthogonal) Lanczos oracle.

The oracle (oracle/bilanczos_oracle.py) builds W_k, V_k and the tridiagonal T_k
of A = 1 - chi0 K from right start chi0 d and left start d in the bilinear form
and reads P_k = beta_1^2 e_1^T T_k^-1 e_1.  These tests tie it to facts that do
not come from its own code:

* the hand-derived two-level closed form (one product: the recursion stops at
  k = 1 with the exact answer);
* on random matrices of the same structure (complex symmetric chi0, real
  symmetric K), at full dimension P_n equals c^T A^-1 b by an LU solve; the
  bases are biorthogonal (W_k^T V_k = I), satisfy A V_k = V_k T_k + beta_{k+1}
  v_{k+1} e_k^T and A^T W_k = W_k T_k + beta_{k+1} w_{k+1} e_k^T, and T_k
  matches the moments c^T A^j b = beta_1^2 (T_k^j)_11 for j = 0 .. 2k-1;
* on the synthetic 4-atom system the recursion converges to the dense LU
  polarizability of chi0_oracle, and its residual estimate equals the true
  residual of x_k = V_k y_k.

Planted mistakes (a dropped three-term coefficient, a sesquilinear instead
of bilinear form, chi0 d as the left start, the last instead of the first
component of y) each fail one of the pins.
"""
import numpy as np
import pytest

import pins
from oracle import bilanczos_oracle as bo
from oracle import chi0_oracle as orc
from paper_1005_5340_amd import synth


def _random_problem(n=8, seed=0):
    """A = 1 - chi K with chi complex symmetric, K real symmetric; b = chi d, c = d."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    chi = 0.3 * (G + G.T) / np.sqrt(n)
    H = rng.standard_normal((n, n))
    K = 0.5 * (H + H.T) / np.sqrt(n)
    A = np.eye(n) - chi @ K
    d = rng.standard_normal(n)
    return A, chi @ d, d


def _a4():
    return synth.make_system("atoms4_orb4", seed=0)


def test_two_level_closed_form():
    two = pins.two_level_system()
    d = two.drives("z")[0]
    for w in (-1.3, 0.0, 0.7, 1.1, 2.0):
        a, rec = bo.polarizability_bilanczos(two, w, d, k_max=5)
        assert rec["alpha"].size == 1 and rec["breakdown"]
        assert abs(a - pins.two_level_alpha(w)) <= 1e-13 * abs(pins.two_level_alpha(w))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_full_dimension_equals_lu(seed):
    A, b, c = _random_problem(8, seed)
    rec = bo.bilanczos(A, b, c, k_max=8)
    ref = c @ np.linalg.solve(A, b)
    assert abs(rec["P"][-1] - ref) <= 1e-10 * abs(ref)


def test_biorthogonality_and_three_term_relations():
    A, b, c = _random_problem(10, 3)
    k = 6
    rec = bo.bilanczos(A, b, c, k_max=k)
    V, W = rec["V"], rec["W"]                # [k + 1, n]
    assert np.max(np.abs(W[:k] @ V[:k].T - np.eye(k))) < 1e-12
    T = bo.tridiagonal(rec["alpha"], rec["beta"][1:])
    e = np.zeros(k); e[-1] = 1.0
    bk = rec["beta"][k]
    assert np.max(np.abs(A @ V[:k].T - V[:k].T @ T - bk * np.outer(V[k], e))) < 1e-12
    assert np.max(np.abs(A.T @ W[:k].T - W[:k].T @ T - bk * np.outer(W[k], e))) < 1e-12


@pytest.mark.parametrize("k", [2, 4, 5])
def test_moment_matching(k):
    A, b, c = _random_problem(9, 4)
    rec = bo.bilanczos(A, b, c, k_max=k)
    T = bo.tridiagonal(rec["alpha"], rec["beta"][1:])
    b1sq = rec["beta"][0] ** 2
    x = b.astype(complex)
    Tp = np.eye(k, dtype=complex)
    for j in range(2 * k):
        m = c @ x
        assert abs(m - b1sq * Tp[0, 0]) <= 1e-10 * max(abs(m), 1e-300), (j, m, b1sq * Tp[0, 0])
        x = A @ x
        Tp = Tp @ T


def test_estimate_matches_recorded_sequence():
    A, b, c = _random_problem(7, 5)
    rec = bo.bilanczos(A, b, c, k_max=5)
    for k in range(1, 6):
        assert abs(bo.estimate(rec["alpha"][:k], rec["beta"][:k]) - rec["P"][k - 1]) < 1e-12 * abs(rec["P"][k - 1])


@pytest.mark.parametrize("omega", [0.05, 0.6, 1.2])
def test_converges_to_lu_polarizability(omega):
    s = _a4()
    d = s.drives("z")[0]
    a, rec = bo.polarizability_bilanczos(s, omega, d, k_max=4000, tol=1e-12)
    ref = orc.polarizability(s, [omega], d[None, :])[0, 0, 0]
    assert rec["res"][-1] <= 1e-12
    assert abs(a - ref) <= 1e-9 * abs(ref)


def test_residual_estimate_is_the_true_residual():
    s = _a4()
    d = s.drives("z")[0]
    chi0 = orc.chi0_matrix(s, 0.6)
    A = orc.response_matrix(s, 0.6, chi0=chi0)
    b = chi0 @ d
    rec = bo.bilanczos(A, b, d, k_max=12)
    k = rec["alpha"].size
    T = bo.tridiagonal(rec["alpha"], rec["beta"][1:])
    y = np.linalg.solve(T, rec["beta"][0] * np.eye(k)[:, 0])
    x = rec["V"][:k].T @ y
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(rec["res"][-1] - true) <= 1e-8 * true


# --------------------------------------------------------------- planted mistakes

def _pins_pass():
    try:
        test_two_level_closed_form()
        for seed in (0, 1, 2):
            test_full_dimension_equals_lu(seed)
        test_biorthogonality_and_three_term_relations()
        for k in (2, 4, 5):
            test_moment_matching(k)
        test_converges_to_lu_polarizability(0.6)
    except AssertionError:
        return False
    return True


def test_pins_pass_unmutated():
    assert _pins_pass()


def _mutant(dropped_three_term=False, sesquilinear=False):
    def run(A, b, c, k_max, tol=0.0):
        A = np.asarray(A, complex); b = np.asarray(b, complex); c = np.asarray(c, complex)
        dot = (lambda x, y: np.vdot(x, y)) if sesquilinear else (lambda x, y: x @ y)
        beta1 = np.sqrt(dot(c, b))
        V, W, al, be, P, res = [b / beta1], [c / beta1], [], [beta1], [], []
        nb = np.linalg.norm(b)
        for k in range(k_max):
            v, w = V[-1], W[-1]
            Av, Atw = A @ v, A.T @ w
            a = dot(w, Av)
            r, s = Av - a * v, Atw - a * w
            if k > 0 and not dropped_three_term:
                r = r - be[k] * V[-2]
                s = s - be[k] * W[-2]
            al.append(a)
            delta = dot(s, r)
            y = bo.solve_tridiagonal(al, be[1:], beta1)
            P.append(beta1 * y[0])
            inv = (np.linalg.norm(r) <= bo.INVARIANT * np.linalg.norm(Av)
                   or np.linalg.norm(s) <= bo.INVARIANT * np.linalg.norm(Atw))
            if delta == 0 or inv:
                be.append(0.0)
                res.append(abs(y[-1]) * np.linalg.norm(r) / nb)
                return dict(alpha=np.array(al), beta=np.array(be), V=np.array(V), W=np.array(W),
                            P=np.array(P), res=np.array(res), breakdown=True)
            bn = np.sqrt(delta)
            be.append(bn)
            V.append(r / bn)
            W.append(s / bn)
            res.append(abs(bn * y[-1]) * np.linalg.norm(V[-1]) / nb)
            if res[-1] <= tol:
                break
        return dict(alpha=np.array(al), beta=np.array(be), V=np.array(V), W=np.array(W),
                    P=np.array(P), res=np.array(res), breakdown=False)
    return run


def test_mutation_dropped_three_term_coefficient(monkeypatch):
    monkeypatch.setattr(bo, "bilanczos", _mutant(dropped_three_term=True))
    assert not _pins_pass()


def test_mutation_sesquilinear_form(monkeypatch):
    monkeypatch.setattr(bo, "bilanczos", _mutant(sesquilinear=True))
    assert not _pins_pass()


def test_mutation_left_start_chi0_d(monkeypatch):
    def wrong(sys, omega, drive, k_max, tol=0.0, eps=None):
        d = np.asarray(drive, float)
        chi0 = orc.chi0_matrix(sys, omega, eps)
        A = orc.response_matrix(sys, omega, eps, chi0)
        rec = bo.bilanczos(A, chi0 @ d, chi0 @ d, k_max, tol)
        return -rec["P"][-1], rec
    monkeypatch.setattr(bo, "polarizability_bilanczos", wrong)
    assert not _pins_pass()


def test_mutation_last_component(monkeypatch):
    real = bo.bilanczos

    def wrong(A, b, c, k_max, tol=0.0):
        rec = real(A, b, c, k_max, tol)
        P = []
        for k in range(1, rec["alpha"].size + 1):
            T = bo.tridiagonal(rec["alpha"][:k], rec["beta"][1:])
            P.append(rec["beta"][0] ** 2 * np.linalg.solve(T, np.eye(k)[:, 0])[-1])
        return dict(rec, P=np.array(P))
    monkeypatch.setattr(bo, "bilanczos", wrong)
    assert not _pins_pass()
