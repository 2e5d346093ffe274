"""Start vectors given by the caller (chi0_solve_opts.x0) on the GPU.

A point starts from the given x0 when its residual is below that of x0 = 0,
else from zero (the rule of the learned warm start).  Checked on the 12-atom
system against the oracle: the exact solution as x0 ends every point before
its first Arnoldi steps; the solution at the neighbouring frequency saves
iterations and gives the oracle's alpha; x0 = 0 is rejected and gives the cold
solve; x0 together with a learned warm start is an error.
"""
import numpy as np
import pytest

import gpu_systems
from oracle import chi0_oracle as orc

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    ctx = chi0.Context(0)
    ctx.set_system_from(sys)
    return torch, chi0, sys, ctx


def test_exact_and_neighbour_start_vectors():
    torch, chi0, sys, ctx = _setup()
    d = sys.drives("xz")
    om = np.linspace(0.05, 1.45, 15)
    kw = dict(restart=sys.n_prod, tol=1e-11, batch=om.size)
    print("[x0] cold solve", flush=True)
    a0, st0, rc0, x = ctx.solve_response(om, sys.eps, d, return_x=True, **kw)
    assert rc0 == 0
    ref = orc.polarizability(sys, om, d)
    # the exact solutions as start vectors: no Arnoldi step is needed
    xo = np.ascontiguousarray(np.stack([orc.solve_response(sys, w, d) for w in om]))
    print("[x0] exact start", flush=True)
    a1, st1, rc1 = ctx.solve_response(om, sys.eps, d, x0=torch.from_numpy(xo).to("cuda"), **kw)
    print(f"[x0] exact start: iterations {st1['iterations'].ravel().tolist()}", flush=True)
    assert rc1 == 0 and st1["iterations"].max() <= 3 and np.all(st1["warm_start"] == 1)
    assert np.abs(a1 - ref).max() <= 1e-9 * np.abs(ref).max()
    # the previous frequency's solution: fewer iterations, the same alpha
    xn = np.ascontiguousarray(np.concatenate([x[:1], x[:-1]]))
    print("[x0] neighbour start", flush=True)
    a2, st2, rc2 = ctx.solve_response(om, sys.eps, d, x0=torch.from_numpy(xn).to("cuda"), **kw)
    assert rc2 == 0
    print(f"[x0] iterations cold {int(st0['iterations'].sum())} neighbour {int(st2['iterations'].sum())}", flush=True)
    assert st2["iterations"].sum() < st0["iterations"].sum()
    assert np.abs(a2 - ref).max() <= 1e-8 * np.abs(ref).max()
    # x0 = 0 is no better than zero: the cold solve (the batches differ in width, so the
    # split-K sums may round differently)
    z = torch.zeros((om.size, 2, sys.n_prod), dtype=torch.complex128, device="cuda")
    a3, st3, rc3 = ctx.solve_response(om, sys.eps, d, x0=z, **kw)
    assert rc3 == 0 and np.all(st3["warm_start"] == 2)
    assert np.abs(a3 - a0).max() <= 1e-10 * np.abs(a0).max()
    assert np.abs(st3["iterations"].astype(int) - st0["iterations"].astype(int)).max() <= 2
    ctx.close()


def test_x0_with_learned_warm_start_is_an_error():
    torch, chi0, sys, ctx = _setup()
    d = sys.drives("z")
    ws = chi0.WarmStart(ctx, np.linspace(0.1, 1.4, 8), sys.eps, d[0], rank=8, width=32, epochs=10,
                        restart=sys.n_prod, batch=8, tol=1e-8)
    z = torch.zeros((2, 1, sys.n_prod), dtype=torch.complex128, device="cuda")
    with pytest.raises(chi0.Chi0Error) as e:
        ctx.solve_response([0.3, 0.6], sys.eps, d, restart=sys.n_prod, warm=ws, x0=z)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        ctx.solve_response([0.3, 0.6], sys.eps, d, x0=torch.zeros((2, 1, 3), dtype=torch.complex128))
    ws.close()
    ctx.close()
