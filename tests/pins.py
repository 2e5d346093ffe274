"""Independent routes that pin the oracle (CPU only, no GPU, no HIP library).

Each route reaches the polarizability or chi0 by a path that shares no
formula with `oracle.chi0_oracle` beyond the paper's definitions, so a
plausible slip in the oracle (a dropped antiresonant term, a flipped sign of
i*eps or of the kernel term, a transposed eigenvector matrix, a lost
occupation factor) shows up as a mismatch in at least one of them.

  * two_level:      a 1-occupied / 1-virtual / 1-product system whose answer
                    follows by hand from eqs. response-mat and sle:
                    alpha(w) = -1 / ((w + i eps)^2 - (D^2 + 2 n D v^2 K)).
  * literal_chi0:   eq. response-mat summed literally over *ordered* pairs
                    (E, F) with the rule E*F < 0 and (n_F - n_E), using the
                    dense N x N vertex of each product and both v^{EF} and
                    v^{FE} (no folding, no support bookkeeping).
  * casida_alpha:   the pole form alpha(w) = sum_I c_I^2 / (w_I - (w+i eps)^2)
                    from the eigen-decomposition of
                    Omega^2 = diag(D^2) + D'^(1/2) Vt^T K Vt D'^(1/2), D' = 2 n D,
                    which follows from eq. eqpolarizability by the push-through
                    identity; it never forms chi0 or solves eq. sle.
  * k0_alpha:       with f = 0, alpha(w) = sum_{EF} 2 n D (d.v)^2 / (D^2 - (w+i eps)^2).
  * asymptote:      alpha(w) (w + i eps)^2 -> -sum_{EF} 2 n D (d.v)^2 as w -> inf,
                    independent of the kernel (the f-sum rule's large-w form).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from paper_1005_5340_amd import synth


# ----------------------------------------------------------------- systems

def custom_system(e, X, atom_orb_offset, prod_atoms, blocks, K, centroids,
                  n_occ, eps, occ_factor=2.0, positions=None):
    """Build a synth.System by hand (used for worked examples)."""
    e = np.asarray(e, float)
    prod_atoms = np.asarray(prod_atoms, np.int32).reshape(-1, 2)
    voff = np.zeros(len(blocks) + 1, np.int64)
    voff[1:] = np.cumsum([np.asarray(b).size for b in blocks])
    vblock = np.concatenate([np.asarray(b, float).ravel() for b in blocks])
    n_atoms = len(atom_orb_offset) - 1
    w = synth.Workload("custom", n_atoms, 0, n_occ, 0, 0, 0.0, 0.0, "whole",
                       eps, 1, 1.0, "z", 10, 1e-10, occ_factor=occ_factor)
    pos = np.zeros((n_atoms, 3)) if positions is None else np.asarray(positions, float)
    return synth.System(workload=w, seed=-1, positions=pos, n_occ=n_occ,
                        occ_factor=occ_factor, eigenvalues=e,
                        X=np.asarray(X, float), atom_orb_offset=np.asarray(atom_orb_offset, np.int32),
                        prod_atoms=prod_atoms, vblock_offset=voff, vblock=vblock,
                        K=np.asarray(K, float).reshape(len(blocks), len(blocks)),
                        centroids=np.asarray(centroids, float).reshape(-1, 3),
                        omegas=np.zeros(1))


TWO_LEVEL = dict(delta=1.0, v=0.5, K=0.25, d=1.0, n=2.0, eps=0.1)


def two_level_system():
    p = TWO_LEVEL
    return custom_system(e=[-p["delta"] / 2, p["delta"] / 2], X=np.eye(2),
                         atom_orb_offset=[0, 2], prod_atoms=[[0, -1]],
                         blocks=[[[0.0, p["v"]], [p["v"], 0.0]]], K=[[p["K"]]],
                         centroids=[[0.0, 0.0, p["d"]]], n_occ=1, eps=p["eps"],
                         occ_factor=p["n"])


def two_level_alpha(omega):
    """Hand-derived closed form for `two_level_system` (see module docstring).

    chi0 = n v^2 [1/(w-D+ie) - 1/(w+D+ie)] = 2 n D v^2 / (z^2 - D^2), z = w + i eps;
    X = chi0 d / (1 - chi0 K) = 2nDv^2 d / (z^2 - D^2 - 2nDv^2 K);  alpha = -d X.
    """
    p = TWO_LEVEL
    z = np.asarray(omega, float) + 1j * p["eps"]
    s = 2 * p["n"] * p["delta"] * p["v"] ** 2
    return -(p["d"] ** 2) * s / (z ** 2 - p["delta"] ** 2 - s * p["K"])


def tiny_workload(eps=0.05, seed_cube=5.0):
    """3 atoms x 3 orbitals, small enough for pure-Python loops."""
    return synth.Workload("tiny3", 3, 3, 4, 2, 2, 4.0, seed_cube, "whole",
                          eps, 8, 1.5, "xyz", 10, 1e-12)


# ------------------------------------------------------- independent routes

def dense_vertices(sys) -> np.ndarray:
    """Each product's vertex scattered into a full N x N matrix: [P, N, N]."""
    N = sys.n_orb
    out = np.zeros((sys.n_prod, N, N))
    off = sys.atom_orb_offset
    for mu in range(sys.n_prod):
        a0, a1 = (int(x) for x in sys.prod_atoms[mu])
        idx = list(range(off[a0], off[a0 + 1]))
        if a1 >= 0:
            idx += list(range(off[a1], off[a1 + 1]))
        s = len(idx)
        o = int(sys.vblock_offset[mu])
        blk = sys.vblock[o:o + s * s].reshape(s, s)
        for i, a in enumerate(idx):
            for j, b in enumerate(idx):
                out[mu, a, b] = blk[i, j]
    return out


def all_pair_vertices(sys) -> np.ndarray:
    """v_mu^{EF} for *all* ordered pairs of MOs: [P, N, N] via einsum."""
    Vd = dense_vertices(sys)
    return np.einsum("aE,mab,bF->mEF", sys.X, Vd, sys.X, optimize=True)


def literal_chi0(sys, omega, eps=None):
    """Eq. response-mat, unfolded, vectorised over (mu, nu) only.

    chi0_{mu nu} = sum_{E,F: e_E e_F < 0} (n_F - n_E) v_mu^{EF} v_nu^{FE} / (w - (e_E - e_F) + i eps)
    """
    eps = sys.eps if eps is None else eps
    v = all_pair_vertices(sys)
    e = sys.eigenvalues
    n = np.where(np.arange(sys.n_orb) < sys.n_occ, sys.occ_factor, 0.0)
    P = sys.n_prod
    chi = np.zeros((P, P), complex)
    for E in range(sys.n_orb):
        for F in range(sys.n_orb):
            if e[E] * e[F] >= 0:
                continue
            w = (n[F] - n[E]) / (omega - (e[E] - e[F]) + 1j * eps)
            chi += w * np.outer(v[:, E, F], v[:, F, E])
    return chi


def literal_chi0_loops(sys, omega, eps=None):
    """Same as `literal_chi0` with every index summed by explicit Python loops."""
    eps = sys.eps if eps is None else eps
    N, P = sys.n_orb, sys.n_prod
    Vd = dense_vertices(sys)
    X = sys.X
    e = sys.eigenvalues
    n = [sys.occ_factor if k < sys.n_occ else 0.0 for k in range(N)]
    nz = [[(a, b) for a in range(N) for b in range(N) if Vd[mu, a, b] != 0.0]
          for mu in range(P)]

    def vtx(mu, E, F):
        s = 0.0
        for a, b in nz[mu]:
            s += X[a, E] * Vd[mu, a, b] * X[b, F]
        return s

    chi = np.zeros((P, P), complex)
    for E in range(N):
        for F in range(N):
            if e[E] * e[F] >= 0:
                continue
            w = (n[F] - n[E]) / (omega - (e[E] - e[F]) + 1j * eps)
            vEF = [vtx(mu, E, F) for mu in range(P)]
            vFE = [vtx(nu, F, E) for nu in range(P)]
            for mu in range(P):
                for nu in range(P):
                    chi[mu, nu] += w * vEF[mu] * vFE[nu]
    return chi


def _folded_parts(sys):
    v = all_pair_vertices(sys)[:, :sys.n_occ, sys.n_occ:]         # [P, No, Nv]
    e = sys.eigenvalues
    D = (e[None, sys.n_occ:] - e[:sys.n_occ, None]).ravel()       # [T]
    Vt = v.reshape(sys.n_prod, -1)                                 # [P, T]
    return Vt, D


def casida_alpha(sys, omegas, drive, eps=None):
    """Pole form of alpha(w) for one drive (no chi0 matrix, no linear solve)."""
    eps = sys.eps if eps is None else eps
    Vt, D = _folded_parts(sys)
    sq = np.sqrt(2.0 * sys.occ_factor * D)
    B = Vt * sq[None, :]
    Om2 = np.diag(D ** 2) + B.T @ sys.K @ B
    w, U = np.linalg.eigh(0.5 * (Om2 + Om2.T))
    c = U.T @ (B.T @ np.asarray(drive, float))
    z2 = (np.asarray(omegas, float) + 1j * eps) ** 2
    return (c[None, :] ** 2 / (w[None, :] - z2[:, None])).sum(1)


def k0_alpha(sys, omegas, drive, eps=None):
    """Closed form with a vanishing kernel."""
    eps = sys.eps if eps is None else eps
    Vt, D = _folded_parts(sys)
    g = Vt.T @ np.asarray(drive, float)
    z2 = (np.asarray(omegas, float) + 1j * eps) ** 2
    return (2 * sys.occ_factor * D[None, :] * g[None, :] ** 2 / (D[None, :] ** 2 - z2[:, None])).sum(1)


def sum_rule_strength(sys, drive):
    """sum_{EF} 2 n D (d.v^{EF})^2, the large-w coefficient of -alpha (w+i eps)^2."""
    Vt, D = _folded_parts(sys)
    g = Vt.T @ np.asarray(drive, float)
    return float((2 * sys.occ_factor * D * g ** 2).sum())


def with_kernel(sys, K):
    return dataclasses.replace(sys, K=np.asarray(K, float))


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
