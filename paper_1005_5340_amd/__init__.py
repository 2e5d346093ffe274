"""MI355X-native iterative TDDFT polarizability (matrix-free chi0 in the dominant-product basis).

Importing the package loads nothing native; the HIP library is loaded by
`paper_1005_5340_amd.chi0` on first use and fails loudly if it is missing.
"""
