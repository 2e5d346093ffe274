"""Planted mistakes in the oracle must be caught by the pins.

Each case replaces one oracle function (on the CPU, through monkeypatch) by a
plausible wrong variant and checks that at least one independent pin from
tests/pins.py now fails.  This guards the pins themselves: a pin suite that
passes a wrong oracle would prove nothing.
"""
import numpy as np
import pytest

import pins
from oracle import chi0_oracle as orc
from paper_1005_5340_amd import synth

_lor = orc.lorentzian
_tv = orc.transition_vertices
_te = orc.transition_energies
_rm = orc.response_matrix
_pol = orc.polarizability


def _checks():
    a4 = synth.make_system("atoms4_orb4", seed=0)
    tiny = synth.make_system(pins.tiny_workload(), seed=3)
    two = pins.two_level_system()
    d = a4.drives("z")[0]
    om = np.linspace(0.0, 1.5, 9)

    def two_level():
        w = np.linspace(-2, 2, 41)
        return pins.rel(orc.polarizability(two, w)[:, 0, 0], pins.two_level_alpha(w)) < 1e-12

    def literal():
        return pins.rel(orc.chi0_matrix(tiny, 0.6), pins.literal_chi0(tiny, 0.6)) < 1e-12

    def casida():
        got = orc.polarizability(a4, om, d[None, :])[:, 0, 0]
        return pins.rel(got, pins.casida_alpha(a4, om, d)) < 1e-10

    def im_positive():
        a = orc.polarizability(a4, om[1:], d[None, :])[:, 0, 0]
        return bool(np.all(a.imag >= 0))

    def conjugation():
        c = orc.chi0_matrix(a4, 0.5)
        return pins.rel(orc.chi0_matrix(a4, -0.5), np.conj(c)) < 1e-13

    return [two_level, literal, casida, im_positive, conjugation]


def m_no_antiresonant(omega, eps, delta, n):
    return n / (omega - delta + 1j * eps)


def m_eps_sign(omega, eps, delta, n):
    return _lor(omega, -eps, delta, n)


def m_no_occupation(omega, eps, delta, n):
    return _lor(omega, eps, delta, 1.0)


def m_transposed_x(sys, occ=None):
    s = synth.System(**{**sys.__dict__, "X": np.ascontiguousarray(sys.X.T)})
    return _tv(s, occ)


def m_wrong_virtual_block(sys, occ=None):
    occ = np.arange(sys.n_occ) if occ is None else np.asarray(occ)
    out = np.empty((sys.n_prod, occ.size, sys.n_orb - sys.n_occ))
    nv = sys.n_orb - sys.n_occ
    for mu in range(sys.n_prod):
        I = sys.support(mu)
        out[mu] = sys.X[np.ix_(I, occ)].T @ sys.vertex(mu) @ sys.X[I, :nv]
    return out


def m_energy_sign(sys):
    return -_te(sys)


def m_kernel_sign(sys, omega, eps=None, chi0=None):
    chi0 = orc.chi0_matrix(sys, omega, eps) if chi0 is None else chi0
    return np.eye(sys.n_prod) + chi0 @ sys.K


def m_alpha_sign(sys, omegas, drives=None, eps=None):
    return -_pol(sys, omegas, drives, eps)


def m_conjugated_dot(sys, omegas, drives=None, eps=None):
    return np.conj(_pol(sys, omegas, drives, eps))


MUTANTS = [
    ("lorentzian", m_no_antiresonant),
    ("lorentzian", m_eps_sign),
    ("lorentzian", m_no_occupation),
    ("transition_vertices", m_transposed_x),
    ("transition_vertices", m_wrong_virtual_block),
    ("transition_energies", m_energy_sign),
    ("response_matrix", m_kernel_sign),
    ("polarizability", m_alpha_sign),
    ("polarizability", m_conjugated_dot),
]


def test_unmutated_oracle_passes_every_check():
    assert all(c() for c in _checks())


@pytest.mark.parametrize("name,fn", MUTANTS, ids=[m[1].__name__ for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(orc, name, fn)
    results = {c.__name__: c() for c in _checks()}
    assert not all(results.values()), f"mutant {fn.__name__} passed every pin: {results}"
