"""Seeded synthetic molecular systems for the iterative polarizability solver.

This module only *draws inputs*: atom positions, Kohn-Sham eigenvalues and LCAO
eigenvectors, the product list with its vertex blocks, the interaction kernel,
the dipole drives and the frequency grid.  It contains none of the response
arithmetic (no chi0, no solve); both the FP64 CPU reference and the HIP path
consume what it produces.

The paper's workloads are real molecules (C60, polythiophene, chlorophyll-a,
PCBM; Sec. 7) computed with SIESTA, which are not available here, so these
synthetic systems stand in for them.  Their structure follows Sec. 3: each
dominant product lives on one atom or on one pair of neighbouring atoms, and
its vertex V^mu_ab is a dense symmetric block over the atomic orbitals of that
atom (pair) and zero elsewhere (eq. vertex-ansatz).  The kernel f_Hxc is a
dense symmetric frequency-independent P x P matrix (Sec. 5).

Recipe (one generator for every size; draw order is part of the contract):
  1. positions: uniform in a cube; minimum spacing 2.5 Bohr, enforced either
     by redrawing the whole configuration ("whole") or atom by atom
     ("sequential", random sequential adsorption);
  2. occupied eigenvalues ~ U[-0.8, -0.2] Ha, then virtual ~ U[0.05, 1.5] Ha,
     each block sorted ascending;
  3. X = Q factor of the QR decomposition of an N(0,1) N x N matrix;
  4. products: `per_atom` on every atom (atom-major), then `per_pair` on every
     atom pair A<B closer than `cutoff` (lexicographic); a pair product's
     support is the union of both atoms' orbitals, A's first;
  5. vertex blocks V^mu ~ N(0, 0.3^2), upper triangle incl. diagonal drawn
     row by row, then mirrored;
  6. K_{mu,nu} = 1/sqrt(|R_mu - R_nu|^2 + 1) - 0.1 delta_{mu,nu}, with R_mu
     the atom position (per-atom product) or the pair midpoint;
  7. drives d_x, d_y, d_z = the centroid coordinates R_mu;
  8. frequencies: inclusive uniform grid on [0, omega_max].
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Dict, List, Optional

import numpy as np
from threadpoolctl import threadpool_limits

__all__ = ["Workload", "System", "WORKLOADS", "make_system", "digest",
           "fingerprint", "same_inputs"]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and solver settings of one synthetic workload."""

    name: str
    n_atoms: int
    orb_per_atom: int
    n_occ: int
    per_atom: int
    per_pair: int
    cutoff: float          # Bohr, strict '<'
    cube: float            # Bohr, side of the placement cube
    placement: str         # "whole" or "sequential"
    eps: float             # Ha, Lorentzian broadening
    n_omega: int
    omega_max: float       # Ha
    drives: str            # subset of "xyz"
    restart: int           # GMRES(m)
    tol: float             # relative residual
    min_spacing: float = 2.5
    occ_lo: float = -0.8
    occ_hi: float = -0.2
    virt_lo: float = 0.05
    virt_hi: float = 1.5
    vertex_sigma: float = 0.3
    kernel_diag_shift: float = -0.1
    occ_factor: float = 2.0


def _cube(n_atoms: int) -> float:
    # Fixed density of 25 Bohr^3 per atom for the larger molecules.
    return float((25.0 * n_atoms) ** (1.0 / 3.0))


WORKLOADS: Dict[str, Workload] = {
    # 4 atoms x 4 orbitals, 6 + 4 products, 64 frequencies: oracle runs in ms.
    "atoms4_orb4": Workload("atoms4_orb4", 4, 4, 8, 6, 4, 4.0, 6.0, "whole",
                            0.02, 64, 1.5, "z", 20, 1e-10),
    # 60 atoms x 9 orbitals (N=540, N_occ=240, ~3.1k products), 128 frequencies.
    "atoms60_orb9": Workload("atoms60_orb9", 60, 9, 240, 15, 8, 5.0, _cube(60),
                             "sequential", 0.01, 128, 1.5, "z", 30, 1e-10),
    # 200 atoms x 9 orbitals (N=1800, N_occ=800, ~12.4k products), 512 x 3 drives.
    "atoms200_orb9": Workload("atoms200_orb9", 200, 9, 800, 15, 8, 5.0, _cube(200),
                              "sequential", 0.01, 512, 2.0, "xyz", 30, 1e-10),
    # 400 atoms x 13 orbitals (N=5200, N_occ=2000, ~40k products), 1024 frequencies.
    "atoms400_orb13": Workload("atoms400_orb13", 400, 13, 2000, 22, 12, 5.0, _cube(400),
                               "sequential", 0.005, 1024, 2.0, "z", 30, 1e-8),
}


@dataclasses.dataclass
class System:
    """One synthetic molecule in the dominant-product representation.

    Arrays (all float64 unless stated):
      positions      [n_atoms, 3]        Bohr
      eigenvalues    [n_orb]             Ha, first n_occ occupied (all < 0 < virtual)
      X              [n_orb, n_orb]      X[a, E] = coefficient of AO a in MO E
      atom_orb_offset[n_atoms+1] int32   AO range of each atom (atom-major AOs)
      prod_atoms     [n_prod, 2] int32   atoms of each product; second = -1 on-site
      vblock_offset  [n_prod+1] int64    start of each product's block in `vblock`
      vblock         [sum s_mu^2]        row-major symmetric s_mu x s_mu blocks
      K              [n_prod, n_prod]    symmetric kernel matrix
      centroids      [n_prod, 3]         product centres R_mu
      omegas         [n_omega]           Ha
    """

    workload: Workload
    seed: int
    positions: np.ndarray
    n_occ: int
    occ_factor: float
    eigenvalues: np.ndarray
    X: np.ndarray
    atom_orb_offset: np.ndarray
    prod_atoms: np.ndarray
    vblock_offset: np.ndarray
    vblock: np.ndarray
    K: np.ndarray
    centroids: np.ndarray
    omegas: np.ndarray

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_orb(self) -> int:
        return int(self.eigenvalues.shape[0])

    @property
    def n_prod(self) -> int:
        return int(self.prod_atoms.shape[0])

    @property
    def eps(self) -> float:
        return self.workload.eps

    def support(self, mu: int) -> np.ndarray:
        """AO indices of product mu's support, in block order."""
        a0, a1 = self.prod_atoms[mu]
        off = self.atom_orb_offset
        idx = list(range(off[a0], off[a0 + 1]))
        if a1 >= 0:
            idx += list(range(off[a1], off[a1 + 1]))
        return np.asarray(idx, dtype=np.int64)

    def vertex(self, mu: int) -> np.ndarray:
        """Product mu's s_mu x s_mu symmetric vertex block (a view)."""
        s = self.support(mu).size
        o = int(self.vblock_offset[mu])
        return self.vblock[o:o + s * s].reshape(s, s)

    def drives(self, which: Optional[str] = None) -> np.ndarray:
        """Dipole drives [n_drive, n_prod] for the given Cartesian letters."""
        which = self.workload.drives if which is None else which
        cols = ["xyz".index(c) for c in which]
        return np.ascontiguousarray(self.centroids[:, cols].T)


def _place_atoms(rng: np.random.Generator, w: Workload) -> np.ndarray:
    n, L, dmin = w.n_atoms, w.cube, w.min_spacing
    if w.placement == "whole":
        for _ in range(100000):
            pos = rng.uniform(0.0, L, size=(n, 3))
            diff = pos[:, None, :] - pos[None, :, :]
            dist = np.sqrt((diff ** 2).sum(-1))
            iu = np.triu_indices(n, 1)
            if dist[iu].min() >= dmin:
                return pos
        raise RuntimeError("atom placement failed")
    if w.placement == "sequential":
        pos = np.empty((n, 3))
        k = 0
        tries = 0
        while k < n:
            p = rng.uniform(0.0, L, size=3)
            tries += 1
            if tries > 1000000:
                raise RuntimeError("atom placement failed")
            if k and np.sqrt(((pos[:k] - p) ** 2).sum(-1)).min() < dmin:
                continue
            pos[k] = p
            k += 1
        return pos
    raise ValueError(w.placement)


def make_system(workload, seed: int = 0) -> System:
    """Draw the synthetic system of `workload` (a name or a Workload)."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    rng = np.random.default_rng(seed)

    pos = _place_atoms(rng, w)
    n_orb = w.n_atoms * w.orb_per_atom
    n_virt = n_orb - w.n_occ
    e_occ = np.sort(rng.uniform(w.occ_lo, w.occ_hi, size=w.n_occ))
    e_virt = np.sort(rng.uniform(w.virt_lo, w.virt_hi, size=n_virt))
    eig = np.concatenate([e_occ, e_virt])
    G = rng.standard_normal((n_orb, n_orb))
    # One BLAS thread: a threaded QR rounds differently with the thread count.
    with threadpool_limits(limits=1):
        X, _ = np.linalg.qr(G)
    X = np.ascontiguousarray(X)

    off = np.arange(w.n_atoms + 1, dtype=np.int32) * w.orb_per_atom

    # Product list: on-site products atom-major, then pair products (A<B).
    prods: List[tuple] = []
    for A in range(w.n_atoms):
        prods += [(A, -1)] * w.per_atom
    for A in range(w.n_atoms):
        d = np.sqrt(((pos[A + 1:] - pos[A]) ** 2).sum(-1))
        for k in np.nonzero(d < w.cutoff)[0]:
            prods += [(A, A + 1 + int(k))] * w.per_pair
    prod_atoms = np.asarray(prods, dtype=np.int32).reshape(-1, 2)
    P = prod_atoms.shape[0]

    sizes = np.where(prod_atoms[:, 1] >= 0, 2, 1).astype(np.int64) * w.orb_per_atom
    voff = np.zeros(P + 1, dtype=np.int64)
    voff[1:] = np.cumsum(sizes * sizes)
    vblock = np.empty(int(voff[-1]))
    for mu in range(P):
        s = int(sizes[mu])
        iu = np.triu_indices(s)
        B = np.zeros((s, s))
        B[iu] = rng.normal(0.0, w.vertex_sigma, size=iu[0].size)
        B = B + np.triu(B, 1).T
        vblock[voff[mu]:voff[mu + 1]] = B.ravel()

    cen = pos[prod_atoms[:, 0]].copy()
    pair = prod_atoms[:, 1] >= 0
    cen[pair] = 0.5 * (pos[prod_atoms[pair, 0]] + pos[prod_atoms[pair, 1]])

    K = np.empty((P, P))
    step = max(1, (1 << 24) // max(P, 1))
    for r0 in range(0, P, step):
        r1 = min(P, r0 + step)
        d2 = ((cen[r0:r1, None, :] - cen[None, :, :]) ** 2).sum(-1)
        K[r0:r1] = 1.0 / np.sqrt(d2 + 1.0)
    K[np.arange(P), np.arange(P)] += w.kernel_diag_shift

    omegas = np.linspace(0.0, w.omega_max, w.n_omega)

    return System(workload=w, seed=seed, positions=pos, n_occ=w.n_occ,
                  occ_factor=w.occ_factor, eigenvalues=eig, X=X,
                  atom_orb_offset=off, prod_atoms=prod_atoms,
                  vblock_offset=voff, vblock=vblock, K=K, centroids=cen,
                  omegas=omegas)


_EXACT = ("positions", "eigenvalues", "atom_orb_offset", "prod_atoms",
          "vblock_offset", "vblock", "K", "centroids", "omegas")


def digest(sys: System, with_x: bool = True) -> str:
    """SHA-256 over the generated arrays (determinism check).

    X comes out of LAPACK, whose last bits may differ between CPU families;
    every other array is drawn or computed elementwise and is bit-stable.
    """
    h = hashlib.sha256()
    for name in _EXACT + (("X",) if with_x else ()):
        a = np.ascontiguousarray(getattr(sys, name))
        h.update(name.encode())
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def fingerprint(sys: System, n_samples: int = 64) -> dict:
    """Digest of the bit-stable arrays plus sampled entries of X.

    Used to check that a stored reference result belongs to the same inputs
    on another machine: the digest must match exactly and the X samples to
    a few ulps.
    """
    r = np.random.default_rng(12345)
    idx = r.integers(0, sys.X.size, size=n_samples)
    return {"workload": sys.workload.name, "seed": sys.seed,
            "digest_no_x": digest(sys, with_x=False),
            "x_index": [int(i) for i in idx],
            "x_value": [float(v) for v in sys.X.ravel()[idx]]}


def same_inputs(sys: System, fp: dict, xtol: float = 1e-12) -> bool:
    """True if `sys` matches a stored `fingerprint` (see above)."""
    if fp.get("digest_no_x") != digest(sys, with_x=False):
        return False
    x = sys.X.ravel()[np.asarray(fp["x_index"], dtype=np.int64)]
    return bool(np.max(np.abs(x - np.asarray(fp["x_value"]))) <= xtol)


def seeded_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex test vectors with N(0,1) real and imaginary parts."""
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)
