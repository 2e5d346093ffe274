"""Plain GMRES with the paper's error estimates, for checking the stopping test.

TEST INFRASTRUCTURE.  Like `chi0_oracle`, this module is a reference for the
tests, the smoke check and the benchmark's CPU-baseline leg only; the product
path never imports it and it shares no code with the HIP library.

Sec. 4.1 of the paper (Koval, Foerster, Coulaud 2010) stops its Krylov
solver on estimates of the relative errors of the solution X and of the
polarizability P = d . X rather than on the relative residual:

    Delta X ~ |A^-1| |r|,      Delta P ~ |A^-1| |d . r|,
    eps_X = Delta X / |X|,     eps_P = Delta P / |P|,

where r is the residual of the current iterate and |A^-1| is the Frobenius
norm of the representation of A^-1 in the Krylov basis.  For GMRES the
iterate of dimension k is x_k = x0 + V_k y_k with y_k the least-squares
solution of H_k y = beta e_1 (H_k the (k+1) x k Hessenberg matrix of the
Arnoldi process), i.e. y_k = pinv(H_k) beta e_1, so the representation of
A^-1 used here is pinv(H_k) (the k x (k+1) map from basis coordinates of the
residual space to those of the solution space).

Everything is computed from its definition at every dimension k: the
Hessenberg matrix by Arnoldi with classical Gram-Schmidt done twice, y_k by a
dense least-squares solve, pinv(H_k) by an SVD, and the residual explicitly
as b - A x_k.  No recurrence, no Givens rotations.
"""
from __future__ import annotations

import numpy as np

__all__ = ["gmres_eps_trace"]


def gmres_eps_trace(A: np.ndarray, b: np.ndarray, d: np.ndarray, kmax: int,
                    x0: np.ndarray | None = None) -> dict:
    """GMRES on A x = b from x0 with eps_X and eps_P at every dimension k = 1..kmax.

    Returns a dict of arrays indexed by k - 1: 'k', 'res' (|r_k| / |b - A x0|),
    'eps_x', 'eps_p', 'ainv_f' (|pinv(H_k)|_F), 'p' (d . x_k), plus 'x' (the
    iterate of the last dimension).  The bilinear product d . x has no
    conjugate (the paper's P = d^mu X_mu).
    """
    A = np.asarray(A, dtype=complex)
    n = A.shape[0]
    b = np.asarray(b, dtype=complex)
    d = np.asarray(d, dtype=complex)
    x0 = np.zeros(n, complex) if x0 is None else np.asarray(x0, dtype=complex)
    r0 = b - A @ x0
    beta = np.linalg.norm(r0)
    kmax = min(kmax, n)
    V = np.zeros((n, kmax + 1), complex)
    H = np.zeros((kmax + 1, kmax), complex)
    V[:, 0] = r0 / beta
    out = {k: [] for k in ("k", "res", "eps_x", "eps_p", "ainv_f", "p")}
    x = x0
    for k in range(1, kmax + 1):
        # Arnoldi step k (eq. orthogonal-krylov-basis, done twice)
        w = A @ V[:, k - 1]
        for _ in range(2):
            h = V[:, :k].conj().T @ w
            w = w - V[:, :k] @ h
            H[:k, k - 1] += h
        H[k, k - 1] = np.linalg.norm(w)
        if H[k, k - 1] > 0:
            V[:, k] = w / H[k, k - 1]
        Hk = H[:k + 1, :k]
        e1 = np.zeros(k + 1, complex)
        e1[0] = beta
        y = np.linalg.lstsq(Hk, e1, rcond=None)[0]
        x = x0 + V[:, :k] @ y
        r = b - A @ x
        ainv = np.linalg.norm(np.linalg.pinv(Hk), "fro")
        P = d @ x
        out["k"].append(k)
        out["res"].append(np.linalg.norm(r) / beta)
        out["eps_x"].append(ainv * np.linalg.norm(r) / np.linalg.norm(x))
        out["eps_p"].append(ainv * abs(d @ r) / abs(P))
        out["ainv_f"].append(ainv)
        out["p"].append(P)
        if H[k, k - 1] == 0:
            break
    res = {key: np.asarray(v) for key, v in out.items()}
    res["x"] = x
    return res
