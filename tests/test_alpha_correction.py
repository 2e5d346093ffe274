"""Residual term of the polarizability (Sec. 4.1), pinned on the CPU.

Sec. 4.1 writes the error of P = d . X as d . A^-1 r for an approximate X
with residual r = chi0 d - A X.  The solver adds this term with A^-T d_k
replaced by d_k + K x_k, which is exact at the solution x_k because chi0
and K are complex symmetric: A^T = 1 - K chi0 and
(1 - K chi0)(d + K x) = d - K chi0 d + K (1 - chi0 K) x = d.  So

    P_ki ~= d_k . x_i + (d_k + K x_k) . r_i

is wrong only to second order in the residuals, where d_k . x_i alone is
wrong to first order.  These tests fix that reading against things other
than the formula itself: the transposed system solved directly by LAPACK,
and the order of the error measured on perturbed solutions of the oracle's
dense system (12-atom system, x/y/z drives, whole 3 x 3 tensor).  A planted
mistake (the Hermitian instead of the bilinear adjoint) must lose the second
order.
"""
import numpy as np
import pytest

import gpu_systems
from oracle import chi0_oracle as orc

OMEGAS = (0.05, 0.6, 1.2)


@pytest.fixture(scope="module")
def dense():
    s = gpu_systems.get("atoms12_orb9")
    D = s.drives("xyz")
    out = []
    for w in OMEGAS:
        chi = orc.chi0_matrix(s, w)
        A = orc.response_matrix(s, w, chi0=chi)
        B = chi @ D.T
        out.append((w, A, B, np.linalg.solve(A, B)))
    return s, D, out


def test_transposed_solution_is_drive_plus_kernel_times_solution(dense):
    s, D, sols = dense
    for w, A, B, X in sols:
        Y = np.linalg.solve(A.T, D.T)            # A^-T d_k by LAPACK, no identity used
        err = np.max(np.abs(Y - (D.T + s.K @ X))) / np.max(np.abs(Y))
        assert err < 1e-9, f"omega={w}: A^-T d differs from d + K x by {err:.2e}"


def _errors(s, D, A, B, X, ts, adjoint):
    """Max relative error of the 3x3 tensor P over perturbed solutions x = x* + t |x*| e."""
    rng = np.random.default_rng(11)
    E = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
    E /= np.linalg.norm(E, axis=0)
    P = D @ X
    plain, corr = [], []
    for t in ts:
        Xp = X + t * E * np.linalg.norm(X, axis=0)
        R = B - A @ Xp
        Pp = D @ Xp
        Pc = Pp + adjoint(D.T + s.K @ Xp).T @ R
        plain.append(np.max(np.abs(Pp - P)) / np.max(np.abs(P)))
        corr.append(np.max(np.abs(Pc - P)) / np.max(np.abs(P)))
    return np.array(plain), np.array(corr)


TS = (1e-4, 1e-5, 1e-6)


def test_residual_term_makes_the_error_second_order(dense):
    s, D, sols = dense
    for w, A, B, X in sols:
        plain, corr = _errors(s, D, A, B, X, TS, adjoint=lambda v: v)
        rp, rc = plain[1:] / plain[:-1], corr[1:] / corr[:-1]
        assert np.all((rp > 0.05) & (rp < 0.2)), f"omega={w}: plain error not first order {plain}"
        assert np.all((rc > 0.005) & (rc < 0.02)), f"omega={w}: corrected error not second order {corr}"
        assert corr[-1] < 1e-2 * plain[-1]


def test_conjugated_adjoint_is_caught(dense):
    """Planted mistake: conj(d + K x) . r (a Hermitian adjoint) keeps a first-order error."""
    s, D, sols = dense
    first_order = 0
    for w, A, B, X in sols:
        _, corr = _errors(s, D, A, B, X, TS, adjoint=np.conj)
        rc = corr[1:] / corr[:-1]
        first_order += int(np.any(rc > 0.05))
    assert first_order >= 2
