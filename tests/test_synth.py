"""The seeded input generator: determinism and the structure of its draws."""
import numpy as np
import pytest

from paper_1005_5340_amd import synth


def test_deterministic_and_seeded():
    a = synth.make_system("atoms4_orb4", seed=0)
    b = synth.make_system("atoms4_orb4", seed=0)
    c = synth.make_system("atoms4_orb4", seed=1)
    assert synth.digest(a) == synth.digest(b)
    assert synth.digest(a) != synth.digest(c)
    fp = synth.fingerprint(a)
    assert synth.same_inputs(b, fp) and not synth.same_inputs(c, fp)


@pytest.mark.parametrize("name", ["atoms4_orb4", "atoms60_orb9"])
def test_structure(name):
    s = synth.make_system(name, seed=0)
    w = s.workload
    N, No = s.n_orb, s.n_occ
    assert N == w.n_atoms * w.orb_per_atom
    e = s.eigenvalues
    assert np.all(e[:No] < 0) and np.all(e[No:] > 0)
    assert np.all(np.diff(e[:No]) >= 0) and np.all(np.diff(e[No:]) >= 0)
    assert e[:No].min() >= w.occ_lo and e[No:].max() <= w.virt_hi
    assert np.allclose(s.X.T @ s.X, np.eye(N), atol=1e-12)
    # minimum spacing and product list
    d = np.sqrt(((s.positions[:, None] - s.positions[None]) ** 2).sum(-1))
    assert d[np.triu_indices(w.n_atoms, 1)].min() >= w.min_spacing
    n_pairs = int((d[np.triu_indices(w.n_atoms, 1)] < w.cutoff).sum())
    assert s.n_prod == w.n_atoms * w.per_atom + n_pairs * w.per_pair
    for mu in range(0, s.n_prod, max(1, s.n_prod // 50)):
        V = s.vertex(mu)
        assert np.array_equal(V, V.T)
        a0, a1 = s.prod_atoms[mu]
        assert V.shape[0] == (2 if a1 >= 0 else 1) * w.orb_per_atom
        if a1 >= 0:
            assert a0 < a1 and d[a0, a1] < w.cutoff
    assert np.array_equal(s.K, s.K.T)
    assert np.allclose(np.diag(s.K), 1.0 + w.kernel_diag_shift)
    assert s.omegas[0] == 0.0 and s.omegas[-1] == w.omega_max and s.omegas.size == w.n_omega
