"""Two-sided (biorthogonal) Lanczos for the polarizability, for checking the library.

TEST INFRASTRUCTURE.  Like `chi0_oracle`, this module is a reference for the
tests, the smoke check and the benchmark's CPU-baseline leg only; the product
path never imports it and it shares no code with the HIP library.

The paper (Koval, Foerster, Coulaud 2010, Sec. 4) notes that the authors had
earlier used an iterative biorthogonal Lanczos method to build an
approximate representation of A = 1 - chi0(w) f that is easy to invert
within its Krylov subspace, before settling on a Krylov solve of eq. sle
followed by P = d.X.  For P(w) = d^T A^-1 chi0 d the biorthogonal form is:

    right start b = chi0 d,  left start c = d,  bilinear form x^T y (no conjugate),
    beta_1 = sqrt(c^T b),  v_1 = b / beta_1,  w_1 = c / beta_1   (w_1^T v_1 = 1),
    for k = 1, 2, ...
        alpha_k   = w_k^T A v_k
        r         = A v_k   - alpha_k v_k - beta_k v_{k-1}
        s         = A^T w_k - alpha_k w_k - beta_k w_{k-1}
        beta_{k+1} = sqrt(s^T r),  v_{k+1} = r / beta_{k+1},  w_{k+1} = s / beta_{k+1}

(v_0 = w_0 = 0).  The bases satisfy W_k^T V_k = I and A V_k = V_k T_k +
beta_{k+1} v_{k+1} e_k^T with T_k the complex symmetric tridiagonal matrix of
diagonal alpha and off-diagonal beta_2..beta_k, so that

    P_k = beta_1^2 e_1^T T_k^-1 e_1,
    x_k = V_k y_k,  T_k y_k = beta_1 e_1,  b - A x_k = -beta_{k+1} (e_k^T y_k) v_{k+1}.

With f = K and chi0 both symmetric, A^T = 1 - K chi0.  Everything here is
written out from those definitions on the dense A.  There is no look-ahead:
an exact zero s^T r, or an r or s that vanishes to rounding (an invariant
subspace: |r| <= 1e-13 |A v_k|), ends the recursion as a breakdown.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from . import chi0_oracle as orc

__all__ = ["bilanczos", "tridiagonal", "solve_tridiagonal", "estimate", "polarizability_bilanczos"]

INVARIANT = 1e-13   # |r| / |A v| (or |s| / |A^T w|) below which the space is taken as invariant


def bilanczos(A: np.ndarray, b: np.ndarray, c: np.ndarray, k_max: int, tol: float = 0.0):
    """Run the recursion on the dense A from right start b and left start c.

    Stops after k_max steps, at a breakdown (s^T r == 0 or an invariant
    subspace), or once the relative
    residual |beta_{k+1} y_k[k]| |v_{k+1}| / |b| is <= tol.  Returns a dict with
    the coefficients alpha [k], beta [k + 1] (beta[0] = beta_1), the bases V, W
    ([k + 1, n] with the last pair v_{k+1}, w_{k+1}), the estimates P [k] and
    relative residuals res [k] after each step, and `breakdown`.
    """
    A = np.asarray(A, dtype=complex)
    b = np.asarray(b, dtype=complex)
    c = np.asarray(c, dtype=complex)
    beta1 = np.sqrt(c @ b)
    V = [b / beta1]
    W = [c / beta1]
    alpha, beta = [], [beta1]
    P, res = [], []
    nb = np.linalg.norm(b)
    breakdown = False
    for k in range(k_max):
        v, w = V[-1], W[-1]
        Av = A @ v
        Atw = A.T @ w
        a = w @ Av
        r = Av - a * v
        s = Atw - a * w
        if k > 0:
            r = r - beta[k] * V[-2]
            s = s - beta[k] * W[-2]
        alpha.append(a)
        delta = s @ r
        bn = np.sqrt(delta)
        y = solve_tridiagonal(alpha, beta[1:], beta1)
        P.append(beta1 * y[0])
        invariant = (np.linalg.norm(r) <= INVARIANT * np.linalg.norm(Av)
                     or np.linalg.norm(s) <= INVARIANT * np.linalg.norm(Atw))
        if delta == 0 or invariant:
            # the residual is r itself (beta_{k+1} v_{k+1} before scaling)
            res.append(abs(y[-1]) * np.linalg.norm(r) / nb)
            beta.append(0.0)
            breakdown = True
            break
        beta.append(bn)
        V.append(r / bn)
        W.append(s / bn)
        res.append(abs(bn * y[-1]) * np.linalg.norm(V[-1]) / nb)
        if res[-1] <= tol:
            break
    return dict(alpha=np.array(alpha), beta=np.array(beta), V=np.array(V), W=np.array(W),
                P=np.array(P), res=np.array(res), breakdown=breakdown)


def tridiagonal(alpha, offdiag) -> np.ndarray:
    """T_k: diagonal alpha (k), symmetric off-diagonal offdiag (k - 1 or more; the first k - 1 used)."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=complex))
    for i in range(k - 1):
        T[i + 1, i] = T[i, i + 1] = offdiag[i]
    return T


def solve_tridiagonal(alpha, offdiag, beta1) -> np.ndarray:
    """y = T_k^-1 (beta_1 e_1) by a banded LU solve (O(k); the dense T_k is not formed)."""
    k = len(alpha)
    ab = np.zeros((3, k), dtype=complex)
    ab[1] = alpha
    ab[0, 1:] = offdiag[:k - 1]
    ab[2, :-1] = offdiag[:k - 1]
    rhs = np.zeros(k, dtype=complex)
    rhs[0] = beta1
    return solve_banded((1, 1), ab, rhs)


def estimate(alpha, beta) -> complex:
    """P_k = beta_1^2 e_1^T T_k^-1 e_1 from the coefficients (beta[0] = beta_1), by a dense solve."""
    k = len(alpha)
    T = tridiagonal(alpha, beta[1:])
    return beta[0] ** 2 * np.linalg.solve(T, np.eye(k)[:, 0])[0]


def polarizability_bilanczos(sys, omega: float, drive, k_max: int, tol: float = 0.0,
                             eps: float | None = None):
    """alpha(w) = -P from the recursion on the dense A(w) of the system (sign reading alpha = -P).

    Returns (alpha, recursion dict).
    """
    d = np.asarray(drive, dtype=float)
    chi0 = orc.chi0_matrix(sys, omega, eps)
    A = orc.response_matrix(sys, omega, eps, chi0)
    rec = bilanczos(A, chi0 @ d, d, k_max, tol)
    return -rec["P"][-1], rec
