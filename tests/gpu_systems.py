"""Seeded synthetic systems used by the GPU parity tests (inputs only)."""
from paper_1005_5340_amd import synth

# 12 atoms x 9 orbitals: N=108 (two 64-row tiles, ragged), N_occ=45 (ragged), P ~ 500.
ATOMS12 = synth.Workload("atoms12_orb9", 12, 9, 45, 15, 8, 5.0, (25.0 * 12) ** (1 / 3),
                         "sequential", 0.01, 16, 1.5, "xyz", 60, 1e-12)
# 8 atoms x 13 orbitals: the widest atom block (13) of the largest workload.
ATOMS8_13 = synth.Workload("atoms8_orb13", 8, 13, 40, 22, 12, 5.0, (25.0 * 8) ** (1 / 3),
                           "sequential", 0.005, 8, 2.0, "z", 60, 1e-12)
# 3 atoms x 3 orbitals.
TINY3 = synth.Workload("tiny3", 3, 3, 4, 2, 2, 4.0, 5.0, "whole", 0.05, 8, 1.5, "xyz", 10, 1e-12)


def get(name, seed=0):
    table = {"atoms12_orb9": ATOMS12, "atoms8_orb13": ATOMS8_13, "tiny3": TINY3}
    return synth.make_system(table.get(name, name), seed)
