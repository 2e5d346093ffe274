"""chi0(w) z on the GPU (HIP path, through the C-ABI) against the FP64 oracle.

Bar: FP64 arithmetic with different summation order, so the normwise
relative difference per right-hand side must stay below 1e-12 (the factored
sequence has ~4 dependent sums over <= a few thousand terms).
"""
import numpy as np
import pytest

import gpu_systems
from oracle import chi0_oracle as orc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


def _ctx(sys):
    from paper_1005_5340_amd import chi0
    c = chi0.Context(0)
    c.set_system_from(sys)
    return c


def _check(torch, ctx, sys, om, seed, tol=1e-12):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((om.size, sys.n_prod)) + 1j * rng.standard_normal((om.size, sys.n_prod))
    out = ctx.apply(om, sys.eps, torch.from_numpy(z).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    worst = 0.0
    for k, w in enumerate(om):
        ref = orc.chi0_apply(sys, float(w), z[k])
        e = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        worst = max(worst, e)
    print(f"[apply] {sys.workload.name} n_rhs={om.size} worst rel err {worst:.2e}", flush=True)
    assert worst < tol


@pytest.mark.parametrize("name", ["atoms4_orb4", "tiny3", "atoms12_orb9", "atoms8_orb13"])
@pytest.mark.parametrize("n_rhs", [1, 2, 5, 40])
def test_apply_matches_oracle(torch, name, n_rhs):
    sys = gpu_systems.get(name)
    ctx = _ctx(sys)
    om = np.linspace(-0.5, 1.6, n_rhs) if n_rhs > 1 else np.array([0.37])
    if n_rhs >= 5:
        om[1] = 0.0
    _check(torch, ctx, sys, om, seed=n_rhs)
    ctx.close()


def test_apply_more_than_one_pass(torch):
    """300 right-hand sides: more than one operator pass (256 per pass)."""
    sys = gpu_systems.get("atoms4_orb4")
    ctx = _ctx(sys)
    om = np.linspace(0.0, 1.5, 300)
    _check(torch, ctx, sys, om, seed=11)
    ctx.close()


def test_apply_reuses_workspace_across_sizes(torch):
    """A large batch then a small one on the same context (stale workspace)."""
    sys = gpu_systems.get("atoms12_orb9")
    ctx = _ctx(sys)
    _check(torch, ctx, sys, np.linspace(0.0, 1.5, 64), seed=1)
    _check(torch, ctx, sys, np.array([0.8]), seed=2)
    _check(torch, ctx, sys, np.linspace(0.1, 0.9, 3), seed=3)
    ctx.close()


def test_apply_full_size_atoms60(torch):
    """Full 60-atom system (N=540, P~3.3k) at sampled frequencies."""
    from paper_1005_5340_amd import synth
    sys = synth.make_system("atoms60_orb9", 0)
    ctx = _ctx(sys)
    _check(torch, ctx, sys, np.array([0.0, 0.61, 1.37]), seed=5)
    ctx.close()


def test_apply_linearity_and_symmetry(torch):
    """chi0(-w) z = conj(chi0(w) conj z) and chi0 is complex symmetric: u.chi0 v = v.chi0 u."""
    sys = gpu_systems.get("atoms12_orb9")
    ctx = _ctx(sys)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(sys.n_prod) + 1j * rng.standard_normal(sys.n_prod)
    v = rng.standard_normal(sys.n_prod) + 1j * rng.standard_normal(sys.n_prod)
    Z = torch.from_numpy(np.stack([u, v, np.conj(u)])).cuda()
    out = ctx.apply(np.array([0.7, 0.7, -0.7]), sys.eps, Z).cpu().numpy()
    assert abs(u @ out[1] - v @ out[0]) < 1e-12 * abs(u @ out[1])
    assert np.linalg.norm(out[2] - np.conj(out[0])) < 1e-12 * np.linalg.norm(out[0])
    ctx.close()


def test_autotuned_tiles_are_bit_identical(torch):
    """Every GEMM tile variant accumulates in the same order: the tuned operator
    equals the untuned (64x64) one bit for bit, also with a variant forced per
    shape by tuning on a size where several are valid (M = P_pad, 128 | M)."""
    from paper_1005_5340_amd import synth
    sys = synth.make_system("atoms60_orb9", 0)
    rng = np.random.default_rng(21)
    om = np.linspace(0.05, 1.4, 48)
    z = rng.standard_normal((om.size, sys.n_prod)) + 1j * rng.standard_normal((om.size, sys.n_prod))
    zt = torch.from_numpy(z).cuda()
    outs = []
    for tune in (False, True, True):
        ctx = _ctx(sys)
        ctx.set_autotune(tune)
        outs.append(ctx.apply(om, sys.eps, zt).cpu().numpy())
        table = ctx.autotune_table()
        if tune:
            print("[autotune]", {k: v["tile"] for k, v in table.items()}, flush=True)
            assert len(table) >= 2 and all(v["us"][v["variant"]] > 0 for v in table.values())
        else:
            assert table == {}
        ctx.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    ctx = _ctx(sys)
    d = sys.drives("z")
    a1, s1, r1 = ctx.solve_response(om[:8], sys.eps, d, restart=sys.n_prod, tol=1e-8, batch=8)
    ctx.set_autotune(False)
    a2, s2, r2 = ctx.solve_response(om[:8], sys.eps, d, restart=sys.n_prod, tol=1e-8, batch=8)
    ctx.close()
    assert r1 == 0 and r2 == 0
    assert np.array_equal(a1, a2) and np.array_equal(s1["iterations"], s2["iterations"])


def test_every_tile_variant_is_bit_identical(torch):
    """Each dense GEMM tile variant forced in turn (where valid for the shape):
    the operator on the 60-atom system and a short batched solve, whose batched
    K V product runs split-K, must equal the 64x64 results bit for bit."""
    from paper_1005_5340_amd import synth
    sys = synth.make_system("atoms60_orb9", 0)
    rng = np.random.default_rng(22)
    om = np.linspace(0.05, 1.4, 40)
    z = rng.standard_normal((om.size, sys.n_prod)) + 1j * rng.standard_normal((om.size, sys.n_prod))
    zt = torch.from_numpy(z).cuda()
    d = sys.drives("z")
    ref_apply = ref_solve = None
    for v in range(6):
        ctx = _ctx(sys)
        ctx.set_autotune(False, force_variant=v)
        out = ctx.apply(om, sys.eps, zt).cpu().numpy()
        a, st, rc = ctx.solve_response(om[:12], sys.eps, d, restart=sys.n_prod, tol=1e-6, batch=12, lanes=1)
        ctx.close()
        assert rc == 0
        print(f"[tiles] variant {v}: iterations {st['iterations'].ravel().tolist()}", flush=True)
        if v == 0:
            ref_apply, ref_solve = out, a
        else:
            assert np.array_equal(out, ref_apply), f"variant {v} changed chi0 z"
            assert np.array_equal(a, ref_solve), f"variant {v} changed the solve"


def test_graph_replays_match_eager():
    """chi0_apply from a HIP graph: every replay, with new vectors written into
    the same buffer and new frequencies, equals the eager call of a second
    context bit for bit (same kernels and tiles); eager work and
    synchronisations run between the replays."""
    import time
    import torch
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    ca, cb = chi0.Context(0), chi0.Context(0)
    ca.set_system_from(sys)
    cb.set_system_from(sys)
    ca.set_graphs(True)
    rng = np.random.default_rng(11)
    nr = 5
    z = torch.zeros((nr, sys.n_prod), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(z)
    for rep in range(6):
        zh = rng.standard_normal((nr, sys.n_prod)) + 1j * rng.standard_normal((nr, sys.n_prod))
        z.copy_(torch.from_numpy(zh))
        om = rng.uniform(0.0, 1.5, nr)
        ca.apply(om, sys.eps, z, out=out)
        ref = cb.apply(om, sys.eps, z)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep} differs"
        ref2 = orc.chi0_apply(sys, om[0], zh[0])
        assert np.max(np.abs(out[0].cpu().numpy() - ref2)) <= 1e-12 * np.max(np.abs(ref2))
        _ = cb.apply(om[::-1].copy(), sys.eps, z)      # eager work between replays
        torch.cuda.synchronize()
    # launch cost: 200 calls with and without the graph on a 4-atom system
    s4 = gpu_systems.get("atoms4_orb4")
    c4 = chi0.Context(0)
    c4.set_system_from(s4)
    z4 = torch.ones((1, s4.n_prod), dtype=torch.complex128, device="cuda")
    o4 = torch.empty_like(z4)
    om4 = np.array([0.7])
    times = {}
    for g in (False, True):
        c4.set_graphs(g)
        for _ in range(3):
            c4.apply(om4, s4.eps, z4, out=o4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(200):
            c4.apply(om4, s4.eps, z4, out=o4)
        torch.cuda.synchronize()
        times[g] = (time.perf_counter() - t0) / 200 * 1e6
    print(f"[graph] 4-atom chi0 apply: {times[False]:.1f} us eager, {times[True]:.1f} us from the graph", flush=True)
    for c in (ca, cb, c4):
        c.close()
