"""The C-ABI library: loads, exports every declared symbol, validates inputs.

CPU only: a host-only context (device -1) runs chi0_set_system's validation
and block-map construction without touching a GPU.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1005_5340_amd import chi0, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    """Every chi0_* function declared in include/*.h (comments stripped)."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, h)).read(), flags=re.S)
            names |= set(re.findall(r"\b(chi0_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(chi0.LIB_PATH):
        pytest.fail("libchi0.so not built (run __graft_entry__.build())")
    return chi0.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_host_only_context_validates_and_sizes(L):
    s = synth.make_system("atoms4_orb4", seed=0)
    with chi0.Context(-1) as ctx:
        ctx.set_system_from(s)
        assert ctx.sizes() == dict(n_orb=16, n_occ=8, n_prod=s.n_prod, n_atoms=4)
        # computing needs a device
        with pytest.raises(chi0.Chi0Error) as e:
            ctx.solve_response([0.1], 0.02, s.drives("z"))
        assert e.value.code == -2


def _args(s):
    return dict(n_atoms=s.n_atoms, positions=s.positions, n_orb=s.n_orb, n_occ=s.n_occ,
                occ_factor=s.occ_factor, eigenvalues=s.eigenvalues.copy(), X=s.X.copy(),
                atom_orb_offset=s.atom_orb_offset.copy(), n_prod=s.n_prod,
                prod_atoms=s.prod_atoms.copy(), vblock_offset=s.vblock_offset.copy(),
                vblock=s.vblock.copy(), K=s.K.copy())


@pytest.mark.parametrize("case,code", [
    ("nan_K", -5), ("inf_vertex", -5), ("asym_K", -6), ("asym_vertex", -6),
    ("unshifted_energy", -1), ("bad_occ", -1), ("bad_offset", -1), ("bad_prod_atom", -1),
    ("bad_vblock_offset", -1), ("occ_factor", -1), ("too_many_orbitals", -1),
])
def test_set_system_error_codes(L, case, code):
    s = synth.make_system("atoms4_orb4", seed=0)
    a = _args(s)
    if case == "nan_K":
        a["K"][1, 2] = np.nan
    elif case == "inf_vertex":
        a["vblock"][5] = np.inf
    elif case == "asym_K":
        a["K"][0, 3] += 1e-6
    elif case == "asym_vertex":
        a["vblock"][1] += 1e-3
    elif case == "unshifted_energy":
        a["eigenvalues"][0] = 0.1
    elif case == "bad_occ":
        a["n_occ"] = s.n_orb
    elif case == "bad_offset":
        a["atom_orb_offset"][2] = a["atom_orb_offset"][1]
    elif case == "bad_prod_atom":
        a["prod_atoms"][3, 1] = a["prod_atoms"][3, 0]
    elif case == "bad_vblock_offset":
        a["vblock_offset"][2] += 1
    elif case == "occ_factor":
        a["occ_factor"] = 0.0
    elif case == "too_many_orbitals":
        a["atom_orb_offset"] = np.array([0, 1, 2, 3, 16], np.int32)
    with chi0.Context(-1) as ctx:
        with pytest.raises(chi0.Chi0Error) as e:
            ctx.set_system(**a)
        assert e.value.code == code, str(e.value)
        assert ctx.last_error


def test_create_rejects_bad_device(L):
    h = C.c_void_p()
    assert L.chi0_create(C.byref(h), -7) == -1
    assert b"device" in L.chi0_last_error(None)


def test_default_options(L):
    o = chi0.SolveOpts()
    L.chi0_solve_opts_default(C.byref(o))
    assert (o.restart, o.max_iter, o.tol, o.precision, o.batch) == (30, 10000, 1e-10, 0, 1)
    assert o.alpha_form == chi0.ALPHA_CORRECTED


def test_timing_filter_on_host_context(L):
    with chi0.Context(-1) as ctx:
        ctx.set_timing(True, only=["dcgs_update", "dcgs_dots"])
        assert ctx.kernel_stats() == {}
        ctx.set_timing(False)
    assert L.chi0_set_timing_filter(None, b"x") == -1


def test_autotune_switch_on_host_context(L):
    with chi0.Context(-1) as ctx:
        ctx.set_autotune(False)
        assert ctx.autotune_table() == {}
        ctx.set_autotune(True)
    assert L.chi0_set_autotune(None, 1) == -1


def test_lanczos_defaults_and_host_context(L):
    o = chi0.LanczosOpts()
    L.chi0_lanczos_opts_default(C.byref(o))
    assert (o.k_max, o.reorth, o.tol, o.check_every, o.n_check, o.graph, o.n_x) == \
        (4000, chi0.LZ_REORTH_PARTIAL, 0.0, 100, 0, 0, 0)
    assert list(o.reserved) == [0, 0]
    s = synth.make_system("atoms4_orb4", seed=0)
    with chi0.Context(-1) as ctx:
        ctx.set_system_from(s)
        with pytest.raises(chi0.Chi0Error) as e:      # host-only: no device to run on
            ctx.lanczos(s.drives("z"), k_max=5)
        assert e.value.code == -2
        res = dict(a=np.ones((1, 2)), b=np.ones((1, 2)), c_norm2=np.ones(1), len=np.array([2], np.int32))
        with pytest.raises(chi0.Chi0Error) as e:
            ctx.lanczos_spectrum(res, [0.5], 0.01)
        assert e.value.code == -2
    assert L.chi0_lanczos(None, 1, None, None, None, None, None, None) == -1


def test_bilanczos_host_context(L):
    s = synth.make_system("atoms4_orb4", seed=0)
    with chi0.Context(-1) as ctx:
        ctx.set_system_from(s)
        with pytest.raises(chi0.Chi0Error) as e:      # host-only: no device to run on
            ctx.solve_bilanczos([0.5], 0.01, s.drives("z"))
        assert e.value.code == -2
    assert L.chi0_solve_bilanczos(None, 1, None, 0.01, 1, None, 1e-10, 10, None, None, None) == -1
