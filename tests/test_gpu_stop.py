"""The paper's stopping test (Sec. 4.1) on the GPU against the GMRES oracle.

With stop = EPS_P the library ends a point when its running estimate
eps_P = |A^-1| |d.r| / |d.x| falls to the tolerance (EPS_PX: eps_X as well),
keeping |A^-1| (the Frobenius norm of R^-1 of the cycle's Hessenberg
factorisation), d.x, |x| and d.r by recurrences over the Arnoldi steps.  The
oracle (oracle/gmres_oracle.py) computes the same estimates from their
definitions at every Krylov dimension on the dense A = 1 - chi0 K.  Checked
per point: the GPU stops at the first dimension where the oracle's estimates
meet the tolerance, reports the oracle's estimates there (1e-6 relative plus
the rounding of the oracle's explicit residual), and returns the oracle's
iterate of that dimension.
"""
import numpy as np
import pytest

import gpu_systems
from oracle import chi0_oracle as orc
from oracle import gmres_oracle as go

pytestmark = pytest.mark.gpu


def _ctx(sys):
    from paper_1005_5340_amd import chi0
    c = chi0.Context(0)
    c.set_system_from(sys)
    return c


@pytest.mark.parametrize("mode,tol", [("eps_p", 1e-2), ("eps_px", 1e-2), ("eps_p", 1e-5), ("eps_px", 1e-4)])
def test_stop_matches_oracle_estimates(mode, tol):
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    om = np.array([0.0, 0.21, 0.5, 0.93, 1.2])
    stop = {"eps_p": chi0.STOP_EPS_P, "eps_px": chi0.STOP_EPS_PX}[mode]
    ctx = _ctx(sys)
    a, st, rc, x = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=tol, batch=om.size,
                                      stop=stop, return_x=True)
    ctx.close()
    assert rc == 0 and st["converged"].all()
    for w in range(om.size):
        k = int(st["iterations"][w, 0]) - 1          # dimension of the stopping step (one-step lag)
        chi0 = orc.chi0_matrix(sys, om[w])
        A = np.eye(sys.n_prod) - chi0 @ sys.K
        b = chi0 @ d[0]
        tr = go.gmres_eps_trace(A, b, d[0], kmax=k + 1)

        def met(i):
            ok = tr["eps_p"][i - 1] <= tol * (1 + 1e-6)
            if mode == "eps_px":
                ok = ok and tr["eps_x"][i - 1] <= tol * (1 + 1e-6)
            return ok

        def missed(i):
            ok = tr["eps_p"][i - 1] > tol * (1 - 1e-6)
            if mode == "eps_px":
                ok = ok or tr["eps_x"][i - 1] > tol * (1 - 1e-6)
            return ok

        print(f"[stop] {mode} tol {tol:g} omega {om[w]:.2f}: k {k} eps_p gpu {st['eps_p'][w, 0]:.6e} "
              f"oracle {tr['eps_p'][k - 1]:.6e}  eps_x gpu {st['eps_x'][w, 0]:.6e} oracle {tr['eps_x'][k - 1]:.6e}"
              f"  true residual {st['rel_residual'][w, 0]:.3e}", flush=True)
        assert k >= 1 and met(k)
        assert all(missed(i) for i in range(1, k))
        xo = tr["x"] if tr["k"][-1] == k else None
        if xo is None:   # the trace ran one dimension further: rebuild the iterate of dimension k
            xo = go.gmres_eps_trace(A, b, d[0], kmax=k)["x"]
        # The oracle forms r = b - A x explicitly, whose rounding is about
        # u |A| |x| per row; the library carries d.r and |r| by recurrences.
        # Tolerance: 1e-6 relative plus four times that rounding carried
        # through the estimate (it dominates once |r| is small).
        u = np.finfo(float).eps
        ax = np.abs(A) @ np.abs(xo)
        ainv = tr["ainv_f"][k - 1]
        bound_p = 4 * ainv * u * (np.abs(d[0]) @ ax) / abs(tr["p"][k - 1])
        bound_x = 4 * ainv * u * np.linalg.norm(ax) / np.linalg.norm(xo)
        assert abs(st["eps_p"][w, 0] - tr["eps_p"][k - 1]) <= 1e-6 * tr["eps_p"][k - 1] + bound_p
        assert abs(st["eps_x"][w, 0] - tr["eps_x"][k - 1]) <= 1e-6 * tr["eps_x"][k - 1] + bound_x
        assert np.linalg.norm(x[w, 0] - xo) <= 1e-8 * np.linalg.norm(xo)
        bound_r = 4 * u * np.linalg.norm(ax) / np.linalg.norm(b)
        assert abs(st["rel_residual"][w, 0] - tr["res"][k - 1]) <= 1e-6 * tr["res"][k - 1] + bound_r


def test_eps_p_stops_no_later_than_combined():
    """eps_P alone stops no later than the combined test; the iterations of the
    three tests at a percent-level tolerance and the error each leaves in P
    (against the exact solve) are reported."""
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get("atoms12_orb9")
    d = sys.drives("z")
    om = np.linspace(0.05, 1.45, 8)
    ctx = _ctx(sys)
    its, errs = {}, {}
    ref = orc.polarizability(sys, om, d)[:, 0, 0]
    for name, stop in (("residual", chi0.STOP_RESIDUAL), ("eps_p", chi0.STOP_EPS_P), ("eps_px", chi0.STOP_EPS_PX)):
        a, st, rc = ctx.solve_response(om, sys.eps, d, restart=sys.n_prod, tol=1e-2, batch=om.size, stop=stop)
        assert rc == 0
        its[name] = st["iterations"][:, 0]
        errs[name] = np.abs(a[:, 0, 0] - ref) / np.abs(ref)
        print(f"[stop] tol 1e-2 {name:8s} iterations {its[name].tolist()} max |P err| / |P| {errs[name].max():.2e}",
              flush=True)
    ctx.close()
    assert np.all(its["eps_p"] <= its["eps_px"])
