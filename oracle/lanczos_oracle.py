"""Krylov (Lanczos) route to the whole spectrum and its poles, for checking the library.

TEST INFRASTRUCTURE.  Like `chi0_oracle`, this module is a reference for the
tests, the smoke check and the benchmark's CPU-baseline leg only; the product
path never imports it and it shares no code with the HIP library.

The paper (Koval, Foerster, Coulaud 2010) computes P(w) frequency by
frequency and names, as further work (Sec. 8), an economical treatment of the
frequency axis that also yields the positions of the poles and the strengths
of their residues.  Written in transition space, the response of Sec. 3 has
the pole form (Casida's equations; in the paper's notation, T = N_occ N_virt
pairs (E occupied, F virtual), D_EF = e_F - e_E, v^{EF} the transition
vertices of eq. response-mat and f the kernel of eq. sle):

    S      = diag(sqrt(2 n D_EF)),
    Om2    = diag(D_EF^2) + S V_t^T f V_t S        (T x T, real symmetric),
    c      = S V_t^T d,
    alpha(w) = c^T (Om2 - (w + i eps)^2)^-1 c,

where V_t is the n_prod x T matrix of v_mu^{EF}.  One Lanczos recursion on
Om2 started from c gives a k x k tridiagonal matrix T_k (diagonal a, off
diagonal b) with

    alpha_k(w) = |c|^2 e_1^T (T_k - (w + i eps)^2)^-1 e_1

for every w at once; the eigenvalues theta_j of T_k approximate the poles of
alpha in (w + i eps)^2 and |c|^2 (u_j)_1^2 their residues.  At k = T (or at an
invariant subspace) the recursion is exact.  The solution of eq. sle itself is
X(w) = -B (Om2 - (w + i eps)^2)^-1 c with B = V_t S (the push-through identity
applied to chi0 = -B diag(D^2 - z)^-1 B^T), which the Krylov basis Q_k
approximates as -|c| B Q_k (T_k - z)^-1 e_1.

Everything here is written out from those definitions: the dense Om2, the
start vector, Lanczos with classical Gram-Schmidt against the whole basis
done twice (full reorthogonalisation), alpha_k by a dense solve with T_k, and
the poles by a dense symmetric eigen-decomposition of T_k.
"""
from __future__ import annotations

import numpy as np

from . import chi0_oracle as co

__all__ = ["casida_parts", "casida_matrix", "start_vector", "lanczos", "spectrum", "poles", "pole_form_solution"]


def casida_parts(sys):
    """S (length T), D^2 (length T) and V_t S (n_prod x T), transitions ordered (E, F) row-major."""
    D = co.transition_energies(sys).ravel()
    S = np.sqrt(2.0 * sys.occ_factor * D)
    Vt = co.transition_vertices(sys).reshape(sys.n_prod, -1)
    return S, D * D, Vt * S[None, :]


def casida_matrix(sys) -> np.ndarray:
    """Dense Om2 = diag(D^2) + (V_t S)^T f (V_t S)."""
    S, D2, B = casida_parts(sys)
    return np.diag(D2) + B.T @ sys.K @ B


def start_vector(sys, drive) -> np.ndarray:
    """c = S V_t^T d for one drive d (length n_prod)."""
    S, D2, B = casida_parts(sys)
    return B.T @ np.asarray(drive, float)


def lanczos(Om2: np.ndarray, c: np.ndarray, k: int, reorth: bool = True, breakdown: float = 1e-12):
    """k steps of the symmetric Lanczos recursion on Om2 from q_1 = c / |c|.

    Returns (a, b, cn2): a[j] = q_j^T Om2 q_j, b[j] = |w_j| the norm of the
    next (unnormalised) vector, cn2 = |c|^2.  With reorth, w_j is projected out
    of every previous q twice (classical Gram-Schmidt, two passes).  Stops
    early, returning shorter arrays, when b[j] <= breakdown * (|a[j]| + b[j-1])
    (an invariant subspace: the recursion is then exact).
    """
    c = np.asarray(c, float)
    cn2 = float(c @ c)
    n = c.size
    k = min(k, n)
    Q = np.zeros((k + 1, n))
    Q[0] = c / np.sqrt(cn2)
    a, b = [], []
    for j in range(k):
        w = Om2 @ Q[j]
        aj = Q[j] @ w
        w = w - aj * Q[j]
        if j > 0:
            w = w - b[-1] * Q[j - 1]
        if reorth:
            for _ in range(2):
                w = w - Q[: j + 1].T @ (Q[: j + 1] @ w)
        bj = float(np.linalg.norm(w))
        a.append(float(aj))
        b.append(bj)
        if bj <= breakdown * (abs(aj) + (b[-2] if j > 0 else 0.0)):
            break
        Q[j + 1] = w / bj
    return np.array(a), np.array(b), cn2


def tridiagonal(a, b) -> np.ndarray:
    """Dense T_k from its diagonal a (length k) and the first k - 1 entries of b."""
    k = len(a)
    T = np.diag(np.asarray(a, float))
    if k > 1:
        off = np.asarray(b[: k - 1], float)
        T += np.diag(off, 1) + np.diag(off, -1)
    return T


def spectrum(a, b, cn2: float, omegas, eps: float) -> np.ndarray:
    """alpha_k(w) = |c|^2 e_1^T (T_k - (w + i eps)^2)^-1 e_1 at each w (dense solves)."""
    T = tridiagonal(a, b)
    k = T.shape[0]
    e1 = np.zeros(k)
    e1[0] = 1.0
    out = np.empty(len(omegas), complex)
    for i, w in enumerate(np.asarray(omegas, float)):
        z = (w + 1j * eps) ** 2
        out[i] = cn2 * np.linalg.solve(T - z * np.eye(k), e1)[0]
    return out


def poles(a, b, cn2: float):
    """Eigenvalues theta of T_k (ascending) and residues |c|^2 (u_j)_1^2."""
    theta, U = np.linalg.eigh(tridiagonal(a, b))
    return theta, cn2 * U[0] ** 2


def pole_form_solution(sys, omega: float, drive, eps: float | None = None) -> np.ndarray:
    """X(w) = -B (Om2 - (w + i eps)^2)^-1 c by a dense solve in transition space."""
    eps = sys.eps if eps is None else eps
    S, D2, B = casida_parts(sys)
    Om2 = np.diag(D2) + B.T @ sys.K @ B
    c = B.T @ np.asarray(drive, float)
    z = (omega + 1j * eps) ** 2
    return -B @ np.linalg.solve(Om2 - z * np.eye(Om2.shape[0]), c)
