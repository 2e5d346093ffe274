"""Pins of the FP64 oracle against closed forms, invariants and literal sums.

None of these tests needs a GPU or the HIP library.  Each compares the
oracle (`oracle.chi0_oracle`) with something the paper's equations or plain
mathematics fix, computed by a route that does not reuse the oracle's code
(see tests/pins.py).
"""
import json
import os

import numpy as np
import pytest

import pins
from oracle import chi0_oracle as orc
from paper_1005_5340_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tiny():
    return synth.make_system(pins.tiny_workload(), seed=3)


@pytest.fixture(scope="module")
def a4():
    return synth.make_system("atoms4_orb4", seed=0)


# --------------------------------------------------------------- worked example

def test_two_level_closed_form():
    """Hand-derived 2-level result (tests/golden/two_level.json)."""
    with open(os.path.join(GOLDEN, "two_level.json")) as f:
        g = json.load(f)
    sys = pins.two_level_system()
    om = np.array([w for w, _, _ in g["values"]])
    ref = np.array([re + 1j * im for _, re, im in g["values"]])
    got = orc.polarizability(sys, om)[:, 0, 0]
    # the stored values are the closed form rounded to 12 significant digits
    assert np.allclose(got, ref, rtol=1e-11, atol=0)
    dense = np.linspace(-3, 3, 601)
    assert pins.rel(orc.polarizability(sys, dense)[:, 0, 0], pins.two_level_alpha(dense)) < 1e-13


def test_two_level_peak_position():
    """Im alpha peaks at the dressed transition sqrt(D^2 + 2nDv^2K) = sqrt(1.25)."""
    sys = pins.two_level_system()
    om = np.linspace(0.9, 1.4, 5001)
    a = orc.polarizability(sys, om)[:, 0, 0]
    wpk = om[np.argmax(a.imag)]
    assert abs(wpk - np.sqrt(1.25)) < 5e-3


# -------------------------------------------------------------- chi0 definition

@pytest.mark.parametrize("omega", [0.0, 0.37, 1.1, -0.6])
def test_chi0_matches_literal_loops(tiny, omega):
    """Folded, chunked oracle chi0 == eq. response-mat summed by explicit loops."""
    ref = pins.literal_chi0_loops(tiny, omega)
    got = orc.chi0_matrix(tiny, omega)
    assert pins.rel(got, ref) < 1e-13


@pytest.mark.parametrize("omega", [0.0, 0.5, 1.3])
def test_chi0_matches_literal_sum(a4, omega):
    ref = pins.literal_chi0(a4, omega)
    assert pins.rel(orc.chi0_matrix(a4, omega), ref) < 1e-13


def test_chi0_identity_eigenvectors():
    """With X = 1 the transition vertex is the vertex element itself."""
    s = synth.make_system(pins.tiny_workload(), seed=4)
    s.X = np.eye(s.n_orb)
    vt = orc.transition_vertices(s)
    Vd = pins.dense_vertices(s)
    assert np.array_equal(vt, Vd[:, :s.n_occ, s.n_occ:])


def test_chi0_symmetries(a4):
    """chi0^T = chi0; chi0(-w) = conj chi0(w) at finite eps; chi0(0) real and <= 0."""
    for w in (0.3, 0.9):
        c = orc.chi0_matrix(a4, w)
        assert pins.rel(c.T, c) < 1e-14
        assert pins.rel(orc.chi0_matrix(a4, -w), np.conj(c)) < 1e-14
    c0 = orc.chi0_matrix(a4, 0.0)
    assert np.max(np.abs(c0.imag)) == 0.0
    ev = np.linalg.eigvalsh(0.5 * (c0.real + c0.real.T))
    assert ev.max() <= 1e-12 * abs(ev).max()


def test_chi0_imaginary_part_sign(a4):
    """For w > 0 every real quadratic form of Im chi0 is <= 0 (absorption)."""
    for w in (0.2, 0.8, 1.4):
        im = orc.chi0_matrix(a4, w).imag
        ev = np.linalg.eigvalsh(0.5 * (im + im.T))
        assert ev.max() <= 1e-12 * abs(ev).max()


def test_chi0_apply_matches_matrix(a4):
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((a4.n_prod, 3)) + 1j * rng.standard_normal((a4.n_prod, 3))
    for w in (0.0, 0.7):
        ref = orc.chi0_matrix(a4, w) @ Z
        assert pins.rel(orc.chi0_apply(a4, w, Z), ref) < 1e-13
        assert pins.rel(orc.chi0_apply(a4, w, Z[:, 1]), ref[:, 1]) < 1e-13


# ----------------------------------------------------------- polarizability

def test_alpha_matches_casida_pole_form(a4):
    d = a4.drives("xyz")
    om = np.linspace(0.0, 1.5, 23)
    got = orc.polarizability(a4, om, d)
    for i in range(3):
        ref = pins.casida_alpha(a4, om, d[i])
        assert pins.rel(got[:, i, i], ref) < 1e-11


def test_alpha_matches_casida_tiny_offdiagonal(tiny):
    """Off-diagonal tensor elements: alpha_xy from the pole form with d_x + d_y."""
    d = tiny.drives("xyz")
    om = np.linspace(0.05, 1.5, 9)
    got = orc.polarizability(tiny, om, d)
    axx = pins.casida_alpha(tiny, om, d[0])
    ayy = pins.casida_alpha(tiny, om, d[1])
    app = pins.casida_alpha(tiny, om, d[0] + d[1])
    axy = 0.5 * (app - axx - ayy)
    assert pins.rel(got[:, 0, 1], axy) < 1e-11
    assert pins.rel(got[:, 1, 0], axy) < 1e-11


def test_alpha_k0_closed_form(a4):
    s = pins.with_kernel(a4, np.zeros_like(a4.K))
    d = s.drives("z")[0]
    om = np.linspace(0.0, 1.5, 31)
    got = orc.polarizability(s, om, d[None, :])[:, 0, 0]
    assert pins.rel(got, pins.k0_alpha(s, om, d)) < 1e-12


def test_alpha_explicit_inverse(a4):
    """Eq. eqpolarizability taken literally: d (1 - chi0 f)^-1 chi0 d, with alpha = -P."""
    d = a4.drives("z")[0]
    for w in (0.0, 0.45, 1.2):
        c = pins.literal_chi0(a4, w)
        Pv = d @ np.linalg.inv(np.eye(a4.n_prod) - c @ a4.K) @ c @ d
        got = orc.polarizability(a4, [w], d[None, :])[0, 0, 0]
        assert abs(got + Pv) <= 1e-11 * abs(Pv)


def test_alpha_large_frequency_limit(a4):
    """alpha (w + i eps)^2 -> -sum 2nD (d.v)^2, the same with and without the kernel."""
    d = a4.drives("z")[0]
    S = pins.sum_rule_strength(a4, d)
    for K in (a4.K, np.zeros_like(a4.K)):
        s = pins.with_kernel(a4, K)
        w = 1e4
        a = orc.polarizability(s, [w], d[None, :])[0, 0, 0]
        assert abs(a * (w + 1j * s.eps) ** 2 + S) < 1e-6 * S


def test_alpha_imaginary_part_nonnegative(a4):
    om = np.linspace(0.0, 1.5, 64)
    a = orc.polarizability(a4, om, a4.drives("xyz"))
    for i in range(3):
        assert np.all(a[1:, i, i].imag >= 0)
    assert np.all(a[0].imag == 0) or np.max(np.abs(a[0].imag)) < 1e-14 * np.max(np.abs(a[0]))


def test_alpha_conjugation_and_reciprocity(a4):
    d = a4.drives("xyz")
    for w in (0.3, 1.1):
        ap = orc.polarizability(a4, [w], d)[0]
        am = orc.polarizability(a4, [-w], d)[0]
        assert pins.rel(am, np.conj(ap)) < 1e-12
        assert pins.rel(ap, ap.T) < 1e-12     # alpha_ki = alpha_ik


def test_alpha_invariances(a4):
    """Product order, sign of each MO and a common permutation leave alpha unchanged."""
    d = a4.drives("z")
    om = [0.2, 0.9]
    ref = orc.polarizability(a4, om, d)
    rng = np.random.default_rng(1)
    s = synth.make_system("atoms4_orb4", seed=0)
    s.X = s.X * rng.choice([-1.0, 1.0], size=s.n_orb)[None, :]
    assert pins.rel(orc.polarizability(s, om, d), ref) < 1e-12
    # permute products: blocks, kernel and drive together
    perm = rng.permutation(a4.n_prod)
    blocks = [a4.vertex(int(m)) for m in perm]
    p = pins.custom_system(a4.eigenvalues, a4.X, a4.atom_orb_offset, a4.prod_atoms[perm],
                           blocks, a4.K[np.ix_(perm, perm)], a4.centroids[perm],
                           a4.n_occ, a4.eps, a4.occ_factor)
    assert pins.rel(orc.polarizability(p, om, d[:, perm]), ref) < 1e-12


def test_residual_norm_of_exact_solution(a4):
    d = a4.drives("z")[0]
    x = orc.solve_response(a4, 0.8, d[None, :])[0]
    assert orc.residual_norm(a4, 0.8, d, x) < 1e-13
    assert orc.residual_norm(a4, 0.8, d, 1.001 * x) > 1e-5


def test_chi0_partial_sums_over_occupied_states_add_up():
    """chi0 restricted to disjoint sets of occupied states (the transitions out of
    each set) adds up to the whole chi0 of eq. response-mat; the sets partition
    the sum over E, so this holds at any frequency."""
    import gpu_systems
    s = gpu_systems.get("atoms12_orb9")
    rng = np.random.default_rng(4)
    perm = rng.permutation(s.n_occ)
    parts = [perm[:7], perm[7:30], perm[30:]]
    for w in (0.0, 0.37):
        full = orc.chi0_matrix(s, w)
        tot = sum(orc.chi0_matrix(s, w, occ_subset=p) for p in parts)
        assert np.max(np.abs(tot - full)) < 1e-12 * np.max(np.abs(full))
        one = orc.chi0_matrix(s, w, occ_subset=parts[0])
        assert np.max(np.abs(one)) > 1e-3 * np.max(np.abs(full))   # a real part of the sum
