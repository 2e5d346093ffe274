"""Lanczos recursion in transition space on the GPU against the oracle.

The library runs the symmetric Lanczos recursion on Om2 = D^2 + S V_t^T K V_t S
with the chi0 operator's kernels (chi0_lanczos) and reads alpha_k(w) off T_k
on the device (chi0_lanczos_spectrum).  Checked against oracle/lanczos_oracle.py
(dense Om2, Lanczos with full reorthogonalisation) and against the dense LU
solve of eq. sle (chi0_oracle):

* at full dimension (k = T on the 4-atom system, all three drives in one
  block) alpha_k equals the LU solve and the poles are eigenvalues of Om2;
* the first coefficients, element by element, on a 12-atom system (ragged
  tiles), with and without reorthogonalisation;
* the converged spectrum against the LU solve to the 1e-6 floored relative
  error of Im alpha, the error measure of the spectrum benchmark, and its ten
  strongest poles against the eigenvalues of the oracle's Om2 and their
  weights (c . u)^2;
* the device continued fraction against the oracle's dense solve with T_k;
* the 60-atom benchmark workload against the stored oracle spectrum;
* the solutions x(w) of eq. sle from the stored basis and the full tensor
  alpha_ki against the LU solve (exact at full dimension, 2e-5 when stopped
  on the spectrum);
* graph replay of the (plain) steps is bit-identical to eager launches;
* the two-level worked example ends after one step (invariant subspace),
  a zero drive gives length 0 and alpha = 0, and bad arguments are errors.
"""
import numpy as np
import pytest

import gpu_systems
import pins
from oracle import chi0_oracle as orc
from oracle import lanczos_oracle as lo
from paper_1005_5340_amd import synth

pytestmark = pytest.mark.gpu


def _ctx(sys):
    from paper_1005_5340_amd import chi0
    c = chi0.Context(0)
    c.set_system_from(sys)
    return c


def _floored_err(got, ref):
    """max_w |Im got - Im ref| / max(|Im ref|, 1e-3 max |Im ref|)."""
    floor = 1e-3 * np.abs(ref.imag).max()
    return float(np.max(np.abs(got.imag - ref.imag) / np.maximum(np.abs(ref.imag), floor)))


def test_full_dimension_three_drives():
    from paper_1005_5340_amd import chi0
    sys = synth.make_system("atoms4_orb4", seed=0)
    T = sys.n_occ * (sys.n_orb - sys.n_occ)
    d = sys.drives("xyz")
    om = sys.omegas
    print(f"[lanczos] atoms4_orb4 full dimension T={T}, 3 drives", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=T, reorth=chi0.LZ_REORTH_FULL)
    alpha = ctx.lanczos_spectrum(res, om, sys.eps)
    ctx.close()
    Om2 = lo.casida_matrix(sys)
    lam = np.linalg.eigvalsh(Om2)
    for s in range(3):
        ref = orc.polarizability(sys, om, d[s][None, :])[:, 0, 0]
        assert pins.rel(alpha[:, s], ref) < 1e-9, s
        k = int(res["len"][s])
        assert 1 <= k <= T
        th, r = chi0.lanczos_poles(res["a"][s, :k], res["b"][s, :k], res["c_norm2"][s])
        heavy = r > 1e-8 * res["c_norm2"][s]
        dist = np.min(np.abs(th[heavy, None] - lam[None, :]), axis=1)
        assert np.all(dist <= 1e-8 * np.abs(lam).max())


# Without reorthogonalisation the recursion loses orthogonality once the first
# Ritz value converges (here the outlying top of the spectrum of Om2, after
# ~9 steps); from then on rounding differences grow and two correct
# implementations produce different coefficients (whose spectra still
# converge), so the plain recursion is compared over its first 8 steps.  Partial
# reorthogonalisation keeps the basis orthogonal only to about sqrt(eps), so its
# coefficients follow the fully reorthogonalised ones to 1e-7.
# A block of three drives and single drives (the operator at three and at one
# column) are both compared.
@pytest.mark.parametrize("reorth,k,tol,drives", [(1, 60, 1e-9, "xyz"), (2, 60, 1e-9, "xyz"), (3, 60, 1e-7, "xyz"),
                                                 (0, 8, 1e-9, "xyz"), (1, 60, 1e-9, "y"), (0, 8, 1e-9, "z")])
def test_coefficients_match_oracle(reorth, k, tol, drives):
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives(drives)
    print(f"[lanczos] atoms12_orb9 coefficients reorth={reorth} k={k} drives={drives}", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=k, reorth=reorth)
    ctx.close()
    Om2 = lo.casida_matrix(sys)
    for s in range(len(drives)):
        c = lo.start_vector(sys, d[s])
        a, b, cn2 = lo.lanczos(Om2, c, k, reorth=bool(reorth))   # the oracle: two passes
        assert int(res["len"][s]) == k
        np.testing.assert_allclose(res["c_norm2"][s], cn2, rtol=1e-12)
        scale = np.abs(a).max()
        assert np.abs(res["a"][s, :k] - a).max() <= tol * scale
        assert np.abs(res["b"][s, :k] - b).max() <= tol * scale


@pytest.mark.parametrize("reorth", [1, 3])
def test_converged_spectrum_meets_benchmark_error(reorth):
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    om = np.linspace(0.0, 1.5, 64)
    print(f"[lanczos] atoms12_orb9 converged spectrum, reorth={reorth}", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=4000, reorth=reorth, tol=1e-9, check_every=50, omega_check=om, eps=sys.eps)
    alpha = ctx.lanczos_spectrum(res, om, sys.eps)[:, 0]
    ctx.close()
    assert res["rc"] == 0
    ref = orc.polarizability(sys, om, d)[:, 0, 0]
    err = _floored_err(alpha, ref)
    print(f"[lanczos] steps {int(res['len'][0])} of T={sys.n_occ * (sys.n_orb - sys.n_occ)}, "
          f"floored Im err {err:.2e}, Re err {pins.rel(alpha.real, ref.real):.2e}", flush=True)
    assert err <= 1e-6
    assert alpha[0].imag == 0.0          # w = 0: z real, the continued fraction is real
    # poles: the strongest ones are converged eigenvalues of Om2, with the
    # weight (c . u)^2 of the oracle's eigenvector
    from paper_1005_5340_amd import chi0
    k = int(res["len"][0])
    th, r = chi0.lanczos_poles(res["a"][0, :k], res["b"][0, :k], res["c_norm2"][0])
    lam, U = np.linalg.eigh(lo.casida_matrix(sys))
    wt = (U.T @ lo.start_vector(sys, d[0])) ** 2
    for idx in np.argsort(r)[::-1][:10]:
        m = np.argmin(np.abs(lam - th[idx]))
        assert abs(lam[m] - th[idx]) <= 1e-9 * np.abs(lam).max(), (th[idx], lam[m])
        assert abs(wt[m] - r[idx]) <= 1e-6 * res["c_norm2"][0], (r[idx], wt[m])


def test_continued_fraction_matches_dense_solve():
    """chi0_lanczos_spectrum (the device continued fraction) against the oracle's dense
    solve with T_k for the same coefficients, three drives, frequencies of both signs."""
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("xyz")
    print("[lanczos] continued fraction vs dense solve", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=200)
    om = np.concatenate([np.linspace(0.0, 2.0, 41), [-0.7, 5.0]])
    got = ctx.lanczos_spectrum(res, om, sys.eps)
    ctx.close()
    for s in range(3):
        k = int(res["len"][s])
        ref = lo.spectrum(res["a"][s, :k], res["b"][s, :k], res["c_norm2"][s], om, sys.eps)
        assert np.abs(got[:, s] - ref).max() <= 1e-11 * np.abs(ref).max(), s


def test_full_size_spectrum_against_stored_reference():
    """The 60-atom workload (T = 72 000) as the benchmark runs it: every point of the
    stored oracle spectrum within 1e-6 (floored Im alpha), and alpha(0) real."""
    import json
    from pathlib import Path
    sys = synth.make_system("atoms60_orb9", seed=0)
    g = json.load(open(Path(__file__).parent / "golden" / "reference_atoms60_orb9_s0.json"))
    assert synth.same_inputs(sys, g["fingerprint"])
    ref = (np.array(g["alpha_re"]) + 1j * np.array(g["alpha_im"]))[:, 0, 0]
    om = sys.omegas[np.asarray(g["omega_index"], int)]
    print("[lanczos] atoms60_orb9 full spectrum", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(sys.drives("z"), k_max=12000, tol=1e-7, check_every=100, omega_check=om, eps=sys.eps)
    alpha = ctx.lanczos_spectrum(res, om, sys.eps)[:, 0]
    ctx.close()
    err = _floored_err(alpha, ref)
    print(f"[lanczos] steps {int(res['len'][0])}, floored Im err {err:.2e}", flush=True)
    assert res["rc"] == 0 and err <= 1e-6
    assert alpha[om == 0.0].imag.tolist() == [0.0] * int((om == 0.0).sum())


def test_solutions_full_dimension():
    """x(w) = -B Q_k y(w) at k = T equals the LU solve of eq. sle, and the full tensor
    alpha_ki = -d_k . x_i equals the oracle's, for three drives in one block."""
    sys = synth.make_system("atoms4_orb4", seed=0)
    T = sys.n_occ * (sys.n_orb - sys.n_occ)
    d = sys.drives("xyz")
    omx = np.array([0.0, 0.3, 0.77, 1.5, -0.4, 0.91])
    from paper_1005_5340_amd import chi0
    print("[lanczos] atoms4_orb4 solutions at full dimension", flush=True)
    ctx = _ctx(sys)
    # full reorthogonalisation: an orthonormal basis to rounding, exact solutions;
    # partial: the basis is orthogonal to about sqrt(eps), and so are the solutions
    for reorth, tol in ((chi0.LZ_REORTH_FULL, 1e-9), (chi0.LZ_REORTH_PARTIAL, 1e-7)):
        res = ctx.lanczos(d, k_max=T, reorth=reorth, eps=sys.eps, omega_x=omx)
        for w, om in enumerate(omx):
            ref = orc.solve_response(sys, om, d)
            for i in range(3):
                assert np.linalg.norm(res["x"][w, i] - ref[i]) <= tol * np.linalg.norm(ref[i]), (reorth, om, i)
        tens = orc.polarizability(sys, omx, d)
        assert np.abs(res["alpha_x"] - tens).max() <= tol * np.abs(tens).max(), reorth
    ctx.close()


def test_solutions_edge_cases():
    """Solutions in several passes with four drives (4 frequencies per pass, the last pass
    ragged), the two-level system (one step), and a zero drive (length 0: x = 0)."""
    from paper_1005_5340_amd import chi0
    sys = synth.make_system("atoms4_orb4", seed=0)
    T = sys.n_occ * (sys.n_orb - sys.n_occ)
    d = np.concatenate([sys.drives("xyz"), np.zeros((1, sys.n_prod))])
    omx = np.array([0.1, 0.45, 0.8, 1.1, 1.3, 1.45])
    print("[lanczos] solution passes with four drives", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=T, reorth=chi0.LZ_REORTH_FULL, eps=sys.eps, omega_x=omx)
    ctx.close()
    assert int(res["len"][3]) == 0
    assert np.all(res["x"][:, 3] == 0) and np.all(res["alpha_x"][:, :, 3] == 0)
    for w, om in enumerate(omx):
        ref = orc.solve_response(sys, om, d[:3])
        for i in range(3):
            assert np.linalg.norm(res["x"][w, i] - ref[i]) <= 1e-9 * np.linalg.norm(ref[i]), (om, i)
    tens = orc.polarizability(sys, omx, d[:3])
    assert np.abs(res["alpha_x"][:, :3, :3] - tens).max() <= 1e-9 * np.abs(tens).max()
    two = pins.two_level_system()
    ctx = _ctx(two)
    om2 = np.linspace(-2, 2, 9)
    r2 = ctx.lanczos(two.drives("z"), k_max=4, eps=two.eps, omega_x=om2)
    ctx.close()
    assert int(r2["len"][0]) == 1
    assert pins.rel(r2["alpha_x"][:, 0, 0], pins.two_level_alpha(om2)) < 1e-13


def test_solutions_converged():
    """On the 12-atom system, stopped on the spectrum: solutions within 2e-5 of the LU
    solve (they converge more slowly than the quadratic form alpha) and the tensor
    within 1e-5 of the oracle's."""
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("xz")
    om = np.linspace(0.0, 1.5, 64)
    omx = np.array([0.0, 0.2, 0.6, 1.3])
    print("[lanczos] atoms12_orb9 solutions", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(d, k_max=4000, tol=1e-9, check_every=50, omega_check=om, eps=sys.eps, omega_x=omx)
    ctx.close()
    assert res["rc"] == 0
    worst = 0.0
    for w, o in enumerate(omx):
        ref = orc.solve_response(sys, o, d)
        for i in range(2):
            worst = max(worst, np.linalg.norm(res["x"][w, i] - ref[i]) / np.linalg.norm(ref[i]))
    tens = orc.polarizability(sys, omx, d)
    terr = np.abs(res["alpha_x"] - tens).max() / np.abs(tens).max()
    print(f"[lanczos] solutions: max rel err {worst:.2e}, tensor err {terr:.2e}", flush=True)
    assert worst <= 2e-5 and terr <= 1e-5


def test_repeated_calls_identical():
    """Two calls on one context, each allocating a 3.9 GB basis (whose zero fill
    must be complete before the recursion writes to it), give the same recursion."""
    sys = synth.make_system("atoms60_orb9", seed=0)
    d = sys.drives("z")
    print("[lanczos] atoms60_orb9 repeated calls, k_max 6000, 300 steps", flush=True)
    ctx = _ctx(sys)
    kw = dict(k_max=6000, tol=1e300, check_every=100, omega_check=[0.5], eps=sys.eps)
    r1 = ctx.lanczos(d, **kw)
    r2 = ctx.lanczos(d, **kw)
    ctx.close()
    for r in (r1, r2):
        assert r["rc"] == 0 and int(r["len"][0]) == 300 and r["c_norm2"][0] > 0
    assert np.array_equal(r1["a"], r2["a"]) and np.array_equal(r1["b"], r2["b"])
    np.testing.assert_allclose(r1["c_norm2"][0], np.sum(lo.start_vector(sys, d[0]) ** 2), rtol=1e-12)


def test_graph_replay_bit_identical():
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("xy")
    print("[lanczos] graph vs eager", flush=True)
    ctx = _ctx(sys)
    eager = ctx.lanczos(d, k_max=150, reorth=0)
    graph = ctx.lanczos(d, k_max=150, reorth=0, graph=True)
    again = ctx.lanczos(d, k_max=150, reorth=0, graph=True)
    ctx.close()
    for r in (graph, again):
        assert np.array_equal(r["a"], eager["a"]) and np.array_equal(r["b"], eager["b"])
        assert np.array_equal(r["len"], eager["len"])


def test_two_level_invariant_subspace_and_zero_drive():
    sys = pins.two_level_system()
    print("[lanczos] two-level system", flush=True)
    ctx = _ctx(sys)
    res = ctx.lanczos(sys.drives("z"), k_max=10)
    assert int(res["len"][0]) == 1
    np.testing.assert_allclose(res["a"][0, 0], 1.25, rtol=1e-14)
    np.testing.assert_allclose(res["c_norm2"][0], 1.0, rtol=1e-14)
    assert res["b"][0, 0] == 0.0
    om = np.linspace(-2, 2, 41)
    got = ctx.lanczos_spectrum(res, om, sys.eps)[:, 0]
    assert pins.rel(got, pins.two_level_alpha(om)) < 1e-13
    z = ctx.lanczos(np.zeros((1, sys.n_prod)), k_max=5)
    assert int(z["len"][0]) == 0 and z["c_norm2"][0] == 0.0
    assert np.all(ctx.lanczos_spectrum(z, om, sys.eps) == 0)
    ctx.close()


def test_errors():
    from paper_1005_5340_amd import chi0
    sys = synth.make_system("atoms4_orb4", seed=0)
    d = sys.drives("z")
    print("[lanczos] error paths", flush=True)
    bare = chi0.Context(0)
    with pytest.raises(chi0.Chi0Error) as e:
        bare.lanczos(d, k_max=5)
    assert e.value.code == -2
    bare.close()
    ctx = _ctx(sys)
    for kw in (dict(k_max=0), dict(reorth=7), dict(tol=1e-6), dict(tol=1e-6, omega_check=[0.5], eps=0.0),
               dict(tol=-1.0)):
        with pytest.raises(chi0.Chi0Error) as e:
            ctx.lanczos(d, **kw)
        assert e.value.code == -1, kw
    for bad in (np.zeros((5, sys.n_prod)), np.zeros((0, sys.n_prod))):
        with pytest.raises(chi0.Chi0Error):
            ctx.lanczos(bad, k_max=5)
    nan = d.copy()
    nan[0, 3] = np.nan
    with pytest.raises(chi0.Chi0Error) as e:
        ctx.lanczos(nan, k_max=5)
    assert e.value.code == -5
    res = ctx.lanczos(d, k_max=5)
    with pytest.raises(chi0.Chi0Error):
        ctx.lanczos_spectrum(res, [0.5], 0.0)
    # a tolerance that k_max steps cannot meet: a warning, coefficients still written
    res = ctx.lanczos(d, k_max=5, tol=1e-300, check_every=1, omega_check=[0.5], eps=sys.eps)
    assert res["rc"] == chi0.NOT_CONVERGED and int(res["len"][0]) == 5
    # solutions need the stored basis
    with pytest.raises(chi0.Chi0Error) as e:
        ctx.lanczos(d, k_max=5, reorth=0, eps=sys.eps, omega_x=[0.5])
    assert e.value.code == -1
    # k_max above the number of transitions is capped to it
    T = sys.n_occ * (sys.n_orb - sys.n_occ)
    res = ctx.lanczos(d, k_max=T + 50)
    assert 1 <= int(res["len"][0]) <= T
    ctx.close()


def test_four_drives_match_single_recursions():
    """A block of four recursions (nc = 4) equals four single ones, coefficient by coefficient."""
    sys = gpu_systems.get("atoms12_orb9")
    d = np.concatenate([sys.drives("xyz"), sys.drives("z") + 0.5 * sys.drives("x")])
    print("[lanczos] four drives in one block", flush=True)
    ctx = _ctx(sys)
    blk = ctx.lanczos(d, k_max=40)
    for s in range(4):
        one = ctx.lanczos(d[s:s + 1], k_max=40)
        assert np.abs(blk["a"][s] - one["a"][0]).max() <= 1e-10 * np.abs(one["a"][0]).max()
        assert np.abs(blk["b"][s] - one["b"][0]).max() <= 1e-10 * np.abs(one["a"][0]).max()
        np.testing.assert_allclose(blk["c_norm2"][s], one["c_norm2"][0], rtol=1e-12)
    ctx.close()


def test_partial_timed_matches_gated():
    """Partial reorthogonalisation decides on the device: the untimed step launches
    the pass every step behind the device flag, the timed step reads the flag and
    launches it only where it runs.  Both give the same recursion bit for bit; the
    timed run counts the executed passes, which is fewer than the steps."""
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("xz")
    print("[lanczos] partial: timed vs gated launches", flush=True)
    ctx = _ctx(sys)
    kw = dict(k_max=600, reorth=chi0.LZ_REORTH_PARTIAL, tol=1e300, check_every=100, omega_check=[0.5],
              eps=sys.eps)
    gated = ctx.lanczos(d, **kw)
    ctx.set_timing(True)
    timed = ctx.lanczos(d, **kw)
    stats = ctx.kernel_stats()
    ctx.set_timing(False)
    ctx.close()
    assert np.array_equal(gated["a"], timed["a"]) and np.array_equal(gated["b"], timed["b"])
    assert np.array_equal(gated["len"], timed["len"])
    steps = int(timed["len"].max())
    npass = stats["lanczos_reorth_dots"]["launches"]
    assert stats["lanczos_omega"]["launches"] == steps
    assert 0 < npass < steps, (npass, steps)
    assert stats["lanczos_reorth_update"]["launches"] == npass
    print(f"[lanczos] {steps} steps, {npass} reorthogonalisation passes", flush=True)


def _simon_decisions(a, b, b_pre):
    """Partial reorthogonalisation decisions from Simon's omega recurrence, replayed
    in NumPy from the recursion's coefficients: w[j+1][i] estimates q_{j+1} . q_i
    from the three-term relation, a pass runs when max |w[j+1][i]| exceeds
    sqrt(eps) (and the step after it too), and a pass resets the row to eps.
    Returns the decisions and the max |w| of each step."""
    eps, thr = np.finfo(float).eps, np.sqrt(np.finfo(float).eps)
    k = b_pre.size
    w_prev, w_cur = np.zeros(k + 2), np.zeros(k + 2)
    w_cur[0] = 1.0
    anorm, carry, out, mxs = 0.0, False, [], []
    for j in range(k):
        aj, bj = a[j], b_pre[j]
        bm = b[j - 1] if j > 0 else 0.0
        an = max(anorm, abs(aj) + bj + bm)
        i = np.arange(j)
        tv = b[i] * w_cur[i + 1] + (a[i] - aj) * w_cur[i] - bm * w_prev[i]
        tv[1:] += b[i[1:] - 1] * w_cur[i[1:] - 1]
        v = (tv + np.where(tv >= 0.0, 1.0, -1.0) * 2.0 * eps * an) / bj
        w_next = np.zeros(k + 2)
        w_next[:j] = v
        w_next[j] = eps * an / bj
        w_next[j + 1] = 1.0
        mx = float(np.max(np.abs(v))) if j else 0.0
        need = carry or mx > thr
        if need:
            w_next[:j + 1] = eps
        carry = (not carry) if need else False
        anorm = an
        out.append(need)
        mxs.append(mx)
        w_prev, w_cur = w_cur, w_next
    return np.array(out), np.array(mxs)


def test_partial_decisions_follow_simons_recurrence():
    """The device-side decision of partial reorthogonalisation (12-atom system, 600
    steps) equals an independent NumPy replay of Simon's recurrence from the
    returned coefficients (and the pre-pass b_j the device used), step by step;
    a first disagreement may only sit at a margin case (|w| within 1e-6 of
    sqrt(eps), where the two evaluation orders can round differently)."""
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    ctx = _ctx(sys)
    ctx.set_timing(True)
    res = ctx.lanczos(d, k_max=600, reorth=chi0.LZ_REORTH_PARTIAL, tol=1e300, check_every=100,
                      omega_check=[0.5], eps=sys.eps)
    ctx.set_timing(False)
    passes, b_pre = ctx.debug_lz_passes(1)
    ctx.close()
    k = int(res["len"][0])
    assert passes.size == k and 0 < passes.sum() < k
    dec, mxs = _simon_decisions(res["a"][0, :k], res["b"][0, :k], b_pre[:, 0])
    same = passes.astype(bool) == dec
    print(f"[lanczos] {k} steps: {int(passes.sum())} device passes, {int(dec.sum())} from the NumPy "
          f"recurrence, {int((~same).sum())} steps differ", flush=True)
    if not same.all():
        j = int(np.argmin(same))
        assert abs(mxs[j] - np.sqrt(np.finfo(float).eps)) <= 1e-6 * np.sqrt(np.finfo(float).eps), (j, mxs[j])
    assert abs(int(passes.sum()) - int(dec.sum())) <= max(2, k // 100)
