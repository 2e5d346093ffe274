"""Mixed precision: low-precision chi0 operators, FP64 iterative refinement and
the relaxed (inexact Krylov) form.

The operator error is bounded by the arithmetic of the orbital transforms
(FP32: 24-bit, split BF16 x 3: ~16-bit operands with FP32 accumulation); the
GMRES-IR and relaxed solves must still reach the FP64 answer because every
cycle ends with an FP64 true residual (the stopping test is unchanged).
"""
import json
import os

import numpy as np
import pytest

import gpu_systems
from oracle import chi0_oracle as orc

pytestmark = pytest.mark.gpu

# normwise relative error bounds of one chi0 application (derived and checked
# against an emulation of the arithmetic in test_mixed_bounds.py: a split
# BF16 product that lost a cross term would be ~60x above its bound), and
# floors that show the reduced arithmetic really ran (FP32 ~3e-7, BF16 x 3
# ~5e-6 observed; an FP64 transform would be ~1e-15)
BOUND = {1: 3e-6, 2: 3e-5}
FLOOR = {1: 1e-9, 2: 1e-7}


def _ctx(sys):
    from paper_1005_5340_amd import chi0
    c = chi0.Context(0)
    c.set_system_from(sys)
    return c


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("name,n_rhs", [("atoms12_orb9", 5), ("atoms8_orb13", 40), ("tiny3", 2)])
def test_low_precision_operator(prec, name, n_rhs):
    import torch
    sys = gpu_systems.get(name)
    ctx = _ctx(sys)
    rng = np.random.default_rng(prec)
    om = np.linspace(0.0, 1.4, n_rhs)
    z = rng.standard_normal((n_rhs, sys.n_prod)) + 1j * rng.standard_normal((n_rhs, sys.n_prod))
    out = ctx.apply(om, sys.eps, torch.from_numpy(z).cuda(), precision=prec).cpu().numpy()
    worst = max(np.linalg.norm(out[k] - orc.chi0_apply(sys, w, z[k])) / np.linalg.norm(orc.chi0_apply(sys, w, z[k]))
                for k, w in enumerate(om))
    print(f"[mixed] {name} prec={prec} worst operator rel err {worst:.2e}", flush=True)
    assert worst < BOUND[prec]
    assert worst > FLOOR[prec]    # really ran in reduced precision
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_iterative_refinement_reaches_fp64(prec):
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    om = np.array([0.0, 0.25, 0.6, 1.05, 1.4])
    ctx = _ctx(sys)
    a, st, rc = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=1e-12, batch=5, precision=prec)
    a64, st64, rc64 = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=1e-12, batch=5)
    ref = orc.polarizability(sys, om, d)
    err = np.max(np.abs(a - ref)) / np.max(np.abs(ref))
    print(f"[mixed] IR prec={prec} err {err:.2e} iters {st['iterations'].ravel().tolist()} "
          f"restarts {st['restarts'].ravel().tolist()} fallback {st['fallback'].ravel().tolist()} "
          f"(fp64 iters {st64['iterations'].ravel().tolist()})", flush=True)
    assert rc == 0 and st["converged"].all()
    assert (st["restarts"] >= 1).all()
    assert err < 1e-9
    ctx.close()


def test_fallback_to_fp64_is_counted_and_exact():
    """A huge inner tolerance makes every low-precision cycle useless; the point
    must fall back to FP64 steps and still converge."""
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    ctx = _ctx(sys)
    a, st, rc = ctx.solve_response([0.7], sys.eps, d, restart=sys.n_prod, tol=1e-12, precision=2,
                                   inner_tol=0.9)
    ref = orc.polarizability(sys, [0.7], d)
    assert rc == 0 and st["converged"][0, 0] == 1
    assert np.max(np.abs(a - ref)) < 1e-9 * np.max(np.abs(ref))
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_relaxed_reaches_fp64_and_switches(prec):
    """One Krylov space: FP64 steps until the residual estimate is small, then the
    reduced-precision operator; the answer is the FP64 one, and both kinds of
    step really ran (counted per point)."""
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    om = np.array([0.0, 0.25, 0.6, 1.05, 1.4])
    ctx = _ctx(sys)
    a, st, rc = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=1e-12, batch=5, precision=prec,
                                   mixed=chi0.MIXED_RELAXED, relax=0.01)
    _, st64, _ = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=1e-12, batch=5)
    ref = orc.polarizability(sys, om, d)
    err = np.max(np.abs(a - ref)) / np.max(np.abs(ref))
    print(f"[mixed] relaxed prec={prec} err {err:.2e} iters {st['iterations'].ravel().tolist()} "
          f"low {st['low_prec_steps'].ravel().tolist()} fallback {st['fallback'].ravel().tolist()}", flush=True)
    assert rc == 0 and st["converged"].all()
    assert err < 1e-9
    assert (st64["low_prec_steps"] == 0).all()
    ok = st["fallback"] == 0
    assert ok.any()
    assert (st["low_prec_steps"][ok] > 0).all()
    assert (st["low_prec_steps"] < st["iterations"]).all()     # FP64 steps first
    ctx.close()


def test_relaxed_bf16x3_atoms60_spectrum_meets_1e6():
    """The 60-atom spectrum (128 frequencies, z drive, residual 1e-10) in the
    relaxed split-BF16 x 3 form: every point within 1e-6 of the oracle's stored
    spectrum in floored Im alpha (the mixed forms' bar)."""
    from paper_1005_5340_amd import chi0, synth
    sys = synth.make_system("atoms60_orb9", 0)
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reference_atoms60_orb9_s0.json")
    rec = json.load(open(gold))
    assert synth.same_inputs(sys, rec["fingerprint"])
    ref = np.array(rec["alpha_re"])[:, 0, 0] + 1j * np.array(rec["alpha_im"])[:, 0, 0]
    ctx = _ctx(sys)
    a, st, rc = ctx.solve_response(sys.omegas, sys.eps, sys.drives("z"), restart=sys.n_prod, tol=1e-10,
                                   batch=128, lanes=1, precision=chi0.PREC_BF16X3, mixed=chi0.MIXED_RELAXED,
                                   relax=0.01)
    ctx.close()
    floor = 1e-3 * np.max(np.abs(ref.imag))
    e = np.abs(a[:, 0, 0].imag - ref.imag) / np.maximum(np.abs(ref.imag), floor)
    low = st["low_prec_steps"].sum() / st["iterations"].sum()
    print(f"[mixed] 60 atoms relaxed BF16x3: max floored Im error {e.max():.2e}, "
          f"{int((e <= 1e-6).sum())}/128 within 1e-6; iterations {int(st['iterations'].sum())}, "
          f"{low:.0%} reduced precision", flush=True)
    assert rc == 0 and st["converged"].all()
    assert (e <= 1e-6).all()
    assert low > 0.1
