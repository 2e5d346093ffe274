#!/usr/bin/env python3
"""Benchmark: absorption-spectrum throughput of the GMRES polarizability solver.

One step = the whole hot path once: solve (1 - chi0(w) K) x = chi0(w) d for
every (frequency, drive) point of the workload's sample and form alpha from
each solution.  The default workload is the 200-atom system (N = 1800,
12.4k products, dense K of 1.2 GB; 512 frequencies on [0, 2] Ha x the x, y, z
drives), solved on the stratified sample of its grid that the stored FP64
oracle reference covers (one frequency per 128-point stratum, x 3 drives).
The timed region covers `--steps` such solves with the system already
resident in HBM.

Printed JSON line (rank 0):
  value      (frequency, drive) points per second whose Im alpha meets the
             bar of their arithmetic against the stored FP64 oracle
             reference (floored relative error: 1e-10 for FP64, 1e-6 with
             low-precision transforms)
  roofline   the kernel with the largest share of GPU time, its algorithmic
             work per launch over its mean launch duration (HIP events on
             the stream it runs on), against the MI355X peak of its bound
  cpu_baseline  the FP64 oracle (dense chi0 + LU) timed on this host's cores
             on a bounded sample of the same workload
  forms      plain (FP64, one point per solve) versus batched, batched +
             mixed precision, batched + mixed + learned warm start, on the
             same points

Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload atoms200_orb9]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X dense peaks: FP64 / FP32 / BF16 matrix cores, HBM3E
PEAK = {"mfma": (78.6e12, "TFLOP/s"), "mfma_f32": (157.3e12, "TFLOP/s"),
        "mfma_bf16": (2.5e15, "TFLOP/s"), "hbm": (8.0e12, "GB/s")}

CHI0_KERNELS = ("vertex_gather", "occ_transform", "virt_transform_lorentz", "virt_back",
                "occ_back", "vertex_contract", "vertex_reduce", "occ_transform_f32",
                "virt_transform_lorentz_f32", "virt_back_f32", "occ_back_f32",
                "virt_transform_lorentz_bf16x3", "virt_back_bf16x3")
MFMA_KERNELS = ("virt_transform_lorentz", "virt_back", "occ_transform", "occ_back", "kernel_matmul",
                "casida_front")
MFMA_F32 = ("virt_transform_lorentz_f32", "virt_back_f32", "occ_transform_f32", "occ_back_f32")
MFMA_BF16 = ("virt_transform_lorentz_bf16x3", "virt_back_bf16x3")


def bound_of(kernel):
    if kernel in MFMA_KERNELS:
        return "mfma"
    if kernel in MFMA_F32:
        return "mfma_f32"
    if kernel in MFMA_BF16:
        return "mfma_bf16"
    return "hbm"


KERNEL_SOURCES = {  # kernel -> source file that defines it (for the counter-staleness check)
    "virt_transform_lorentz": "kernels_gemm.hip", "virt_back": "kernels_gemm.hip",
    "kernel_matmul": "kernels_gemm.hip", "kernel_matvec": "kernels_gemm.hip",
    "occ_transform": "kernels_gemm.hip", "occ_back": "kernels_gemm.hip",
    "vertex_gather": "kernels_vertex.hip", "vertex_contract": "kernels_vertex.hip",
    "vertex_reduce": "kernels_vertex.hip",
    "lanczos_reorth_dots": "kernels_lanczos.hip", "lanczos_reorth_update": "kernels_lanczos.hip",
    "casida_front": "kernels_gemm.hip",
}


def im_errors(a, ref):
    floor = 1e-3 * np.max(np.abs(ref.imag))
    return np.abs(a.imag - ref.imag) / np.maximum(np.abs(ref.imag), floor)


def source_sha(kernel):
    f = os.path.join(ROOT, "paper_1005_5340_amd", "csrc", KERNEL_SOURCES.get(kernel, "kernels_krylov.hip"))
    return hashlib.sha256(open(f, "rb").read()).hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counters, or None if absent or stale."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha") != source_sha(kernel):
        return None
    return rec.get("bytes_per_launch")


def cpu_info():
    """Host CPU model name and logical core count (for the oracle baseline)."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count()}


def cpu_baseline(sys_, drives, n_sample, seed=0):
    """The FP64 oracle (dense chi0 + LU) timed on this host.  Small systems: whole
    frequencies (n_sample seeded grid points).  Large ones, where one frequency takes
    tens of minutes: at one seeded grid frequency, the dense chi0 restricted to a few
    occupied states (transitions out of them) and the whole LU solve of eq. sle for
    every drive with it; the chi0 build is linear in the occupied states, so a
    frequency costs n_occ / k times the partial build plus the solve."""
    from threadpoolctl import threadpool_info
    from oracle import chi0_oracle as orc
    rng = np.random.default_rng(seed)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()
                   if p.get("user_api") == "blas"] or [1])
    info = {"unit": "spectrum points/s", "cores": int(threads), "kind": "oracle",
            "blas_threads": int(threads), **cpu_info()}
    if sys_.n_prod <= 4000:
        idx = np.sort(rng.choice(sys_.omegas.size, size=n_sample, replace=False))
        t0 = time.perf_counter()
        for k in idx:
            orc.polarizability(sys_, [sys_.omegas[k]], drives)
        dt = time.perf_counter() - t0
        pts = n_sample * drives.shape[0]
        return {"value": pts / dt, **info,
                "sample": f"{n_sample} of {sys_.omegas.size} frequencies x {drives.shape[0]} drive(s) "
                          f"(grid indices {idx.tolist()}), dense chi0 + LU in FP64, {dt:.1f} s"}
    k_occ = 5
    wi = int(rng.integers(sys_.omegas.size))
    w = float(sys_.omegas[wi])
    occ = np.arange(k_occ)
    t0 = time.perf_counter()
    chi = orc.chi0_matrix(sys_, w, occ_subset=occ)
    t_chi = time.perf_counter() - t0
    t0 = time.perf_counter()
    A = orc.response_matrix(sys_, w, chi0=chi)
    np.linalg.solve(A, chi @ drives.T)
    t_solve = time.perf_counter() - t0
    del chi, A
    t_freq = t_chi * sys_.n_occ / k_occ + t_solve
    return {"value": drives.shape[0] / t_freq, **info,
            "seconds_per_frequency": t_freq,
            "sample": f"grid frequency {wi} (omega {w:.4f}): dense chi0 over the transitions of {k_occ} of "
                      f"{sys_.n_occ} occupied states ({t_chi:.1f} s) and the LU solve of eq. sle for "
                      f"{drives.shape[0]} drive(s) ({t_solve:.1f} s); per frequency "
                      f"{sys_.n_occ // k_occ} x the partial chi0 + the solve = {t_freq:.0f} s (extrapolated)"}


def chi0_flops(s):
    """Table t:flops count of one chi0 z (complex z, real X and vertices)."""
    N, No = s.n_orb, s.n_occ
    Nv = N - No
    S_V = int(sum(s.support(m).size for m in range(s.n_prod)))   # sum of product supports
    return 8.0 * No * S_V + 8.0 * N * No * Nv + 6.0 * No * Nv


def apply_only(a, s, ctx):
    """chi0.v GFLOP/s: REPS applications of chi0(w_r) to a batch of seeded vectors."""
    import torch
    from paper_1005_5340_amd import chi0
    rng = np.random.default_rng(7)
    nb = a.batch
    om = s.omegas[rng.choice(s.omegas.size, size=nb, replace=nb > s.omegas.size)]
    z = torch.tensor(rng.standard_normal((nb, s.n_prod)) + 1j * rng.standard_normal((nb, s.n_prod)),
                     dtype=torch.complex128, device="cuda")
    F = chi0_flops(s)
    res = {}
    ref = None
    for name, prec in (("fp64", chi0.PREC_FP64), ("fp32", chi0.PREC_FP32), ("bf16x3", chi0.PREC_BF16X3)):
        if a.precision != "fp64" and name not in ("fp64", a.precision):
            continue
        out = ctx.apply(om, s.eps, z, precision=prec)    # first call tunes the GEMM tiles
        torch.cuda.synchronize()
        ctx.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(a.apply_only):
            ctx.apply(om, s.eps, z, out=out, precision=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.apply_only
        ks = ctx.kernel_stats()
        ctx.set_timing(False)
        if ref is None:
            ref = out.clone()
        err = float((torch.linalg.vector_norm(out - ref, dim=1) / torch.linalg.vector_norm(ref, dim=1)).max())
        kern = {k: {"ms_per_apply": v["ms"] / a.apply_only,
                    "rate": (v["flops"] / 1e12 if bound_of(k) != "hbm" else v["bytes"] / 1e9) / (v["ms"] * 1e-3),
                    "unit": "TFLOP/s" if bound_of(k) != "hbm" else "GB/s"} for k, v in ks.items()}
        dom = max(ks, key=lambda k: ks[k]["ms"])
        b = bound_of(dom)
        peak, unit = PEAK[b]
        work = ks[dom]["bytes"] if b == "hbm" else ks[dom]["flops"]
        res[name] = {"gflops": F * nb / dt / 1e9, "ms_per_apply": dt * 1e3,
                     "max_rel_diff_vs_fp64_gpu": err,
                     "dominant": {"kernel": dom, "achieved": work / (ks[dom]["ms"] * 1e-3) / (1e9 if b == "hbm" else 1e12),
                                  "peak": peak / (1e9 if b == "hbm" else 1e12), "unit": unit,
                                  "frac": work / (ks[dom]["ms"] * 1e-3) / peak},
                     "kernels": kern}
        print(f"[bench] apply {name}: {res[name]['gflops']:.0f} GFLOP/s, {dt * 1e3:.2f} ms per batch of {nb}",
              file=sys.stderr, flush=True)
    print(json.dumps({"metric": "chi0.v GFLOP/s (Table t:flops count)", "value": res["fp64"]["gflops"],
                      "unit": "GFLOP/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                      "config": {"workload": a.workload, "seed": a.seed, "n_orb": s.n_orb, "n_occ": s.n_occ,
                                 "n_prod": s.n_prod, "batch": nb, "reps": a.apply_only},
                      "flops_per_apply": F, "precisions": res}), flush=True)
    ctx.close()


def lanczos_mode(a, s, ctx, drives, drive_letters, omegas, grid, ref, ref_idx, ref_drive):
    """One step = one Lanczos recursion per drive (up to 4 in a block) until the spectrum on the
    grid has converged, then alpha on the grid from the continued fraction."""
    import torch
    from paper_1005_5340_amd import chi0
    reorth = (chi0.LZ_REORTH_NONE if a.lz_plain else
              chi0.LZ_REORTH_FULL if a.lz_full else chi0.LZ_REORTH_PARTIAL)

    def run(graph=True):
        res = ctx.lanczos(drives, k_max=a.lz_kmax, reorth=reorth, tol=a.lz_tol, check_every=a.lz_check,
                          omega_check=omegas, eps=s.eps, graph=graph and reorth == chi0.LZ_REORTH_NONE)
        return res, ctx.lanczos_spectrum(res, omegas, s.eps)

    print(f"[bench] lanczos {a.workload}: T={s.n_occ * (s.n_orb - s.n_occ)} drives={drive_letters} "
          f"points={omegas.size * drives.shape[0]} tol={a.lz_tol:g} reorth={reorth}",
          file=sys.stderr, flush=True)
    ks_all = {}
    if not a.no_timing:     # breakdown: eager launches, every kernel timed
        ctx.set_timing(True)
        t0 = time.perf_counter()
        run(graph=False)
        ks_all = ctx.kernel_stats()
        ctx.set_timing(False)
        print(f"[bench] breakdown run (eager, all kernels timed) {time.perf_counter() - t0:.3f} s",
              file=sys.stderr, flush=True)
    for i in range(a.warmup):
        t0 = time.perf_counter()
        run()
        print(f"[bench] warmup {i} {time.perf_counter() - t0:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        res, alpha = run()
        print(f"[bench] step {i} done: {res['len'].tolist()} steps, rc {res['rc']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    npts = omegas.size * drives.shape[0]
    if a.dump_alpha:
        np.save(a.dump_alpha, alpha)
    acc = {"checked": False}
    passing = npts
    if ref is not None and np.all(np.isin(ref_idx, grid)):
        diag = alpha[np.searchsorted(grid, ref_idx)]
        rdiag = np.stack([ref[:, ref_drive[i], ref_drive[i]] for i in range(drives.shape[0])], 1)
        err = np.stack([im_errors(diag[:, i], rdiag[:, i]) for i in range(drives.shape[0])], 1)
        full = ref_idx.size == grid.size
        passing = int((err <= 1e-6).sum()) if full else npts * float((err <= 1e-6).mean())
        acc = {"checked": True, "max_im_rel_err": float(err.max()), "median_im_rel_err": float(np.median(err)),
               "max_re_rel_err": float(np.max(np.abs(diag.real - rdiag.real) / np.abs(rdiag.real))),
               "points_passing_1e-6": int((err <= 1e-6).sum()), "points_checked": int(err.size)}
    roof = None
    if ks_all:
        tot = sum(v["ms"] for v in ks_all.values())
        dom = max(ks_all, key=lambda k: ks_all[k]["ms"])
        rec = ks_all[dom]
        bound = bound_of(dom)
        peak, unit = PEAK[bound]
        work = rec["bytes"] if bound == "hbm" else rec["flops"]
        scale = 1e9 if bound == "hbm" else 1e12
        traffic = load_traffic(dom, a.workload) if reorth != chi0.LZ_REORTH_NONE else None
        roof = {"kernel": dom, "bound": "hbm" if bound == "hbm" else "mfma",
                "achieved": work / (rec["ms"] * 1e-3) / scale, "peak": peak / scale, "unit": unit,
                "frac": work / (rec["ms"] * 1e-3) / peak, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                "traffic_over_algorithmic": (traffic / (rec["bytes"] / rec["launches"])) if traffic and rec["bytes"] else None,
                "launches": rec["launches"], "mean_launch_us": 1e3 * rec["ms"] / rec["launches"],
                "share_of_gpu_time": rec["ms"] / tot,
                "note": "from the eager breakdown run (every kernel timed)"}
        print("[bench] kernel            launches   ms   share", file=sys.stderr)
        for k, v in sorted(ks_all.items(), key=lambda kv: -kv[1]["ms"]):
            print(f"[bench] {k:30s} {int(v['launches']):8d} {v['ms']:9.2f} {100 * v['ms'] / tot:6.1f}%",
                  file=sys.stderr)
    sol = None
    if a.lz_solutions and not a.lz_plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = ctx.lanczos(drives, k_max=a.lz_kmax, reorth=reorth, tol=a.lz_tol, check_every=a.lz_check,
                         omega_check=omegas, eps=s.eps, omega_x=omegas)
        t_all = time.perf_counter() - t0
        diag_x = np.stack([rs["alpha_x"][:, i, i] for i in range(drives.shape[0])], 1)
        sol = {"seconds_with_recursion": t_all, "seconds_solutions": t_all - dt, "n_x": int(omegas.size),
               "max_rel_diff_alpha_x_vs_continued_fraction": float(np.max(np.abs(diag_x - alpha)) /
                                                                    np.max(np.abs(alpha)))}
        if acc.get("checked"):
            dx = diag_x[np.searchsorted(grid, ref_idx)]
            ex = np.stack([im_errors(dx[:, i], rdiag[:, i]) for i in range(drives.shape[0])], 1)
            sol["max_im_rel_err_alpha_x"] = float(ex.max())
        print(f"[bench] solutions at {omegas.size} frequencies: {t_all:.3f} s with the recursion",
              file=sys.stderr, flush=True)
    # poles and residues of the first drive's recursion (host, after the timed region)
    k0 = int(res["len"][0])
    t0 = time.perf_counter()
    th, rr = chi0.lanczos_poles(res["a"][0, :k0], res["b"][0, :k0], res["c_norm2"][0])
    t_poles = time.perf_counter() - t0
    top = np.argsort(rr)[::-1][:5]
    poles = {"k": k0, "seconds": t_poles, "c_norm2": float(res["c_norm2"][0]),
             "with_residue_above_1e-6_of_c_norm2": int((rr > 1e-6 * res["c_norm2"][0]).sum()),
             "negative": int((th < 0).sum()),
             "strongest": [{"theta": float(th[i]), "excitation_energy": float(np.sqrt(th[i])) if th[i] > 0 else None,
                            "residue": float(rr[i])} for i in top]}
    out = {
        "metric": "spectrum points/s at 1e-6 rel err in Im alpha vs FP64 oracle",
        "value": passing / dt, "unit": "spectrum points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": a.workload, "seed": a.seed, "method": "lanczos (transition space)",
                   "n_orb": s.n_orb, "n_occ": s.n_occ, "n_prod": s.n_prod, "n_omega": int(omegas.size),
                   "drives": drive_letters, "eps": s.eps, "points": npts, "k_max": a.lz_kmax, "tol": a.lz_tol,
                   "check_every": a.lz_check,
                   "reorth": "none" if a.lz_plain else "full" if a.lz_full else "partial"},
        "lanczos_steps": res["len"].tolist(), "lanczos_rc": int(res["rc"]),
        "us_per_lanczos_step": dt * 1e6 / max(int(res["len"].max()), 1),
        "accuracy": acc, "roofline": roof, "cpu_baseline": None, "poles": poles, "solutions": sol,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def measure_forms(a, s, ctx, omegas, grid, drives, drive_letters, ref, ref_idx, ref_drive, restart, tol,
                  batched, alpha64):
    """The method's forms on the points of the timed steps, each timed by the wall
    clock over one solve with the kernel timer off, then solved again with every
    kernel timed (HIP events on every launch) for its dominant kernel:
    plain = FP64, one point per solve (the paper's order of work); batched = the
    timed steps; batched + mixed = split-BF16x3 transforms, relaxed; batched +
    mixed + warm = the same with a learned warm start, one network per drive
    (each fitted on `--forms-train` seeded frequencies of its drive's plain FP64
    solutions).  Points pass at 1e-10 (FP64) or 1e-6 (mixed) in floored Im alpha
    against the stored oracle reference; where none is stored (400 atoms), against
    the timed steps' FP64 solve at the same tolerance (alpha64), and the FP64 forms
    are not checked."""
    import torch
    from paper_1005_5340_amd import chi0
    F = chi0_flops(s)
    nd = drives.shape[0]

    def errs(alpha, dsel, fp64=False):
        if ref is None:
            if fp64:
                return None
            d = np.stack([alpha[:, i, i] for i in range(len(dsel))], 1)
            rd = np.stack([alpha64[:, j, j] for j in dsel], 1)
            return np.stack([im_errors(d[:, i], rd[:, i]) for i in range(len(dsel))], 1)
        d = np.stack([alpha[:, i, i] for i in range(len(dsel))], 1)[np.searchsorted(grid, ref_idx)]
        rd = np.stack([ref[:, ref_drive[j], ref_drive[j]] for j in dsel], 1)
        return np.stack([im_errors(d[:, i], rd[:, i]) for i in range(len(dsel))], 1)

    def solve_timed(calls):
        """calls: list of (drive indices, solve kwargs); one solve_response per entry.
        Solved twice: wall-clock time with the kernel timer off (as in the timed
        steps), then the per-kernel record with every launch timed."""
        def once():
            return [(dsel, ctx.solve_response(omegas, s.eps, drives[dsel], restart=restart, max_iter=a.max_iter,
                                              tol=tol, lanes=1, **kw)) for dsel, kw in calls]
        ctx.set_timing(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = once()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ctx.set_timing(True)
        once()
        torch.cuda.synchronize()
        ks = ctx.kernel_stats()
        ctx.set_timing(False)
        return res, sec, ks

    def record(res, sec, ks, bar, note):
        e = [errs(al, dsel, bar < 1e-8) for dsel, (al, st, rc) in res]
        its = np.concatenate([st["iterations"].ravel() for _, (al, st, rc) in res])
        apps = sum(int((st["iterations"] + st["restarts"] + 1).sum()) for _, (al, st, rc) in res)
        npts = sum(al.shape[0] * len(dsel) for dsel, (al, st, rc) in res)
        passing = npts if e[0] is None else int(sum((x <= bar).sum() for x in e))
        chi0_ms = sum(ks[k]["ms"] for k in CHI0_KERNELS if k in ks)
        dom = max(ks, key=lambda k: ks[k]["ms"])
        b = bound_of(dom)
        peak, unit = PEAK[b]
        work = ks[dom]["bytes"] if b == "hbm" else ks[dom]["flops"]
        sc = 1e9 if b == "hbm" else 1e12
        rec = {"points_per_s": passing / sec, "seconds": sec, "passing": passing, "bar": bar, "points": npts,
               "max_im_rel_err": None if e[0] is None else float(max(x.max() for x in e)),
               "iterations": {"mean": float(its.mean()), "max": int(its.max()), "total": int(its.sum()),
                              "reduced_precision": int(sum(st["low_prec_steps"].sum() for _, (al, st, rc) in res))},
               "converged": int(sum(st["converged"].sum() for _, (al, st, rc) in res)),
               "chi0_tflops": F * apps / (chi0_ms * 1e-3) / 1e12 if chi0_ms > 0 else None,
               "dominant": {"kernel": dom, "achieved": work / (ks[dom]["ms"] * 1e-3) / sc, "peak": peak / sc,
                            "unit": unit, "frac": work / (ks[dom]["ms"] * 1e-3) / peak,
                            "share_of_gpu_time": ks[dom]["ms"] / sum(v["ms"] for v in ks.values())},
               "note": note}
        print(f"[bench] form: {note}: {rec['points_per_s']:.3f} points/s, {passing}/{npts} within {bar:g}, "
              f"{sec:.2f} s, mean iterations {rec['iterations']['mean']:.0f}", file=sys.stderr, flush=True)
        return rec

    alld = list(range(nd))
    relax = a.relax or 0.01
    mixed = dict(precision=chi0.PREC_BF16X3, mixed=chi0.MIXED_RELAXED, relax=relax)
    out = {}
    r, sec, ks = solve_timed([(alld, dict(batch=1))])
    out["plain"] = record(r, sec, ks, 1e-10, "plain: FP64, one point per solve")
    out["batched"] = batched
    r, sec, ks = solve_timed([(alld, dict(batch=a.batch, **mixed))])
    out["batched_mixed"] = record(r, sec, ks, 1e-6, "batched + split-BF16x3 transforms (relaxed, switch at "
                                                     f"{relax:g} tol |b| / u)")
    # learned warm start: one network per drive, fitted on plain FP64 solutions
    rng = np.random.default_rng(1000)
    om_train = np.sort(rng.uniform(a.band_lo, float(s.omegas.max()), a.forms_train))
    t0 = time.perf_counter()
    nets = [chi0.WarmStart(ctx, om_train, s.eps, drives[i], rank=min(64, a.forms_train), width=256,
                           epochs=3000, restart=restart, batch=min(a.forms_train, a.batch), tol=tol)
            for i in alld]
    t_fit = time.perf_counter() - t0
    r, sec, ks = solve_timed([(alld, dict(batch=a.batch, warm=nets, **mixed))])
    rw = record(r, sec, ks, 1e-6, "batched + split-BF16x3 (relaxed) + learned warm start (a network per drive)")
    st = r[0][1][1]
    it0 = out["batched_mixed"]["iterations"]["total"]   # the same points, no warm start
    rw.update(warm_fit_seconds=t_fit, warm_train_frequencies=a.forms_train,
              warm_used=int((st["warm_start"] == 1).sum()), warm_rejected=int((st["warm_start"] == 2).sum()),
              median_rel_residual_of_x0=float(np.median(st["warm_rel0"])),
              iterations_without_warm=it0, iterations_with_warm=int(st["iterations"].sum()))
    out["batched_mixed_warm"] = rw
    for n in nets:
        n.close()
    return out


def spectrum_range(a, s, ctx, drives, ref, ref_idx, ref_drive):
    """The grid points lo..hi-1 of the workload's whole grid (--spectrum-range lo:hi),
    every drive, unrestarted GMRES at the workload tolerance, in chunks of frequencies
    solved as one batch each: 4 frequencies below 0.3 Ha (points there need up to ~10^4
    iterations), 32 above; one line per chunk.  alpha goes to --dump-alpha (.npz) and is
    checked against every stored oracle frequency in the range."""
    import torch
    nw = s.omegas.size
    lo, hi = (int(v) for v in a.spectrum_range.split(":"))
    if not 0 <= lo < hi <= nw:
        raise SystemExit(f"--spectrum-range must satisfy 0 <= lo < hi <= {nw}")
    idx = np.arange(lo, hi)
    chunks, k = [], 0
    while k < idx.size:
        n = 4 if s.omegas[idx[k]] < 0.3 else 32
        chunks.append(idx[k:k + n])
        k += n
    nd = drives.shape[0]
    alpha = np.zeros((idx.size, nd, nd), complex)
    iters = np.zeros((idx.size, nd), int)
    conv = np.zeros((idx.size, nd), int)
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for c in chunks:
        t0 = time.perf_counter()
        al, st, _ = ctx.solve_response(s.omegas[c], s.eps, drives, restart=s.n_prod, tol=a.tol or s.workload.tol,
                                       batch=min(96, nd * c.size), max_iter=s.n_prod, lanes=1)
        sel = c - idx[0]
        alpha[sel], iters[sel], conv[sel] = al, st["iterations"], st["converged"]
        print(f"[bench] chunk omega[{c[0]}..{c[-1]}] ({s.omegas[c[0]]:.3f}-{s.omegas[c[-1]]:.3f} Ha): "
              f"{time.perf_counter() - t0:.1f} s, iterations max {st['iterations'].max()} mean "
              f"{st['iterations'].mean():.0f}, converged {int(st['converged'].sum())}/{st['converged'].size}",
              file=sys.stderr, flush=True)
    sec = time.perf_counter() - t_all
    if a.dump_alpha:
        np.savez(a.dump_alpha, idx=idx, alpha=alpha, iters=iters, conv=conv, seconds=sec)
    acc = None
    if ref is not None:
        errs = []
        for n, kref in enumerate(ref_idx):
            if kref in idx:
                al = alpha[kref - idx[0]]
                for i in range(nd):
                    fl = 1e-3 * np.max(np.abs(ref[:, ref_drive[i], ref_drive[i]].imag))
                    r0 = ref[n, ref_drive[i], ref_drive[i]]
                    errs.append(abs(al[i, i].imag - r0.imag) / max(abs(r0.imag), fl))
        acc = {"oracle_points": len(errs), "max_im_rel_err": float(max(errs)) if errs else None}
    pos = s.omegas[idx] > 0
    scale = float(np.max(np.abs(alpha)))
    checks = {"max_asymmetry_rel": float(np.max(np.abs(alpha - np.swapaxes(alpha, 1, 2)))) / scale,
              "min_im_alpha_diag_over_max": float(min(alpha[pos, i, i].imag.min() for i in range(nd))) / scale
              if pos.any() else None}
    print(json.dumps({"spectrum_range": [lo, hi], "workload": a.workload, "points": int(idx.size * nd),
                      "seconds": sec, "points_per_s": idx.size * nd / sec, "converged": int(conv.sum()),
                      "iterations": {"mean": float(iters.mean()), "max": int(iters.max()), "total": int(iters.sum())},
                      "accuracy": acc, "checks": checks}), flush=True)
    ctx.close()


def warm_experiment(a, s, ctx, drives, restart, tol):
    """Learned warm start against the zero start and the previous-frequency start on
    one drive: `--warm` seeded training frequencies (uniform on [--band-lo, omega_max],
    seed 1000) give the network (plain FP64 solves at the test tolerance); the
    `--omega-sample` test frequencies are evenly spaced grid points of the same band.
    Each start solves the test points once, batched, in the requested precision; the
    zero-start solve judges the others' error (the plain solve at the same tolerance).
    The previous-frequency start uses the solution at the next lower grid point,
    solved first (its cost is reported apart)."""
    import torch
    from paper_1005_5340_amd import chi0
    d = drives[:1]
    prec = {"fp64": chi0.PREC_FP64, "fp32": chi0.PREC_FP32, "bf16x3": chi0.PREC_BF16X3}[a.precision]
    kw = dict(restart=restart, max_iter=a.max_iter, tol=tol, batch=a.batch, precision=prec, lanes=1,
              mixed=chi0.MIXED_RELAXED if a.mixed == "relaxed" else chi0.MIXED_REFINE, relax=a.relax)
    band = s.omegas >= a.band_lo
    gi = np.flatnonzero(band)
    test = gi[np.round(np.linspace(1, gi.size - 1, a.omega_sample)).astype(int)]
    om = s.omegas[test]
    rng = np.random.default_rng(1000)
    om_train = np.sort(rng.uniform(a.band_lo, float(s.omegas.max()), a.warm))
    out = {"workload": a.workload, "drive": a.drives or "first", "tol": tol, "precision": a.precision,
           "mixed": a.mixed, "restart": restart, "max_iter": a.max_iter, "test_grid_indices": test.tolist(),
           "train_frequencies": om_train.tolist()}

    def solve(name, **extra):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        al, st, rc = ctx.solve_response(om, s.eps, d, **kw, **extra)
        torch.cuda.synchronize()
        r = {"seconds": time.perf_counter() - t0, "iterations": int(st["iterations"].sum()),
             "max_iterations": int(st["iterations"].max()), "converged": int(st["converged"].sum()),
             "alpha": al[:, 0, 0]}
        print(f"[bench] warm experiment: {name}: {r['seconds']:.1f} s, iterations {r['iterations']} "
              f"(max {r['max_iterations']}), converged {r['converged']}/{om.size}", file=sys.stderr, flush=True)
        return r, st

    zero, _ = solve("zero start")
    t0 = time.perf_counter()
    ws = chi0.WarmStart(ctx, om_train, s.eps, d[0], rank=min(64, a.warm), width=256, epochs=3000,
                        restart=restart, batch=min(a.warm, a.batch), tol=tol)
    t_fit = time.perf_counter() - t0
    print(f"[bench] warm experiment: network fitted in {t_fit:.1f} s", file=sys.stderr, flush=True)
    learned, stl = solve("learned start", warm=ws)
    ws.close()
    t0 = time.perf_counter()
    _, _, _, xp = ctx.solve_response(s.omegas[test - 1], s.eps, d, return_x=True, **kw)
    t_prev = time.perf_counter() - t0
    x0 = torch.from_numpy(np.ascontiguousarray(xp)).to("cuda")
    prev, stp = solve("previous-frequency start", x0=x0)
    ref = zero["alpha"]
    floor = 1e-3 * np.max(np.abs(ref.imag))
    for name, r, st in (("zero_start", zero, None), ("learned", learned, stl), ("previous_frequency", prev, stp)):
        al = r.pop("alpha")
        r["max_im_rel_diff_vs_zero_start"] = float(np.max(np.abs(al.imag - ref.imag) /
                                                        np.maximum(np.abs(ref.imag), floor)))
        r["saved_vs_zero_start"] = 1.0 - r["iterations"] / zero["iterations"]
        if st is not None:
            r["median_rel_residual_of_x0"] = float(np.median(st["warm_rel0"]))
            r["rejected"] = int((st["warm_start"] == 2).sum())
        out[name] = r
    out["learned"]["fit_seconds"] = t_fit
    out["previous_frequency"]["seconds_neighbour_solves"] = t_prev
    print(json.dumps(out), flush=True)
    ctx.close()


def bilanczos_mode(a, s, ctx, drives, drive_letters, omegas, grid, ref, ref_idx, ref_drive, tol):
    """One step = the two-sided Lanczos solve of every (omega, drive) point (chi0_solve_bilanczos);
    afterwards, untimed, the GMRES solve of the same points for comparison."""
    import torch
    npts = omegas.size * drives.shape[0]

    def run():
        return ctx.solve_bilanczos(omegas, s.eps, drives, tol=tol, max_steps=a.bl_max_steps)

    print(f"[bench] two-sided lanczos {a.workload}: {npts} points, tol {tol:g}", file=sys.stderr, flush=True)
    ks_all = {}
    if not a.no_timing:
        ctx.set_timing(True)
        run()
        ks_all = ctx.kernel_stats()
        ctx.set_timing(False)
    for _ in range(a.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        alpha, steps, status, rc = run()
        print(f"[bench] step {i} done: steps mean {steps.mean():.0f} max {steps.max()}, rc {rc}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    acc = {"checked": False}
    passing = npts
    if ref is not None and np.all(np.isin(ref_idx, grid)):
        diag = alpha[np.searchsorted(grid, ref_idx)]
        rdiag = np.stack([ref[:, ref_drive[i], ref_drive[i]] for i in range(drives.shape[0])], 1)
        err = np.stack([im_errors(diag[:, i], rdiag[:, i]) for i in range(drives.shape[0])], 1)
        full = ref_idx.size == grid.size
        passing = int((err <= 1e-6).sum()) if full else npts * float((err <= 1e-6).mean())
        acc = {"checked": True, "max_im_rel_err": float(err.max()), "median_im_rel_err": float(np.median(err)),
               "points_passing_1e-6": int((err <= 1e-6).sum()), "points_passing_1e-10": int((err <= 1e-10).sum()),
               "points_checked": int(err.size)}
    roof = None
    if ks_all:
        tot = sum(v["ms"] for v in ks_all.values())
        dom = max(ks_all, key=lambda k: ks_all[k]["ms"])
        rec = ks_all[dom]
        bound = bound_of(dom)
        peak, unit = PEAK[bound]
        work = rec["bytes"] if bound == "hbm" else rec["flops"]
        scale = 1e9 if bound == "hbm" else 1e12
        roof = {"kernel": dom, "bound": "hbm" if bound == "hbm" else "mfma",
                "achieved": work / (rec["ms"] * 1e-3) / scale, "peak": peak / scale, "unit": unit,
                "frac": work / (rec["ms"] * 1e-3) / peak, "traffic": None,
                "launches": rec["launches"], "mean_launch_us": 1e3 * rec["ms"] / rec["launches"],
                "share_of_gpu_time": rec["ms"] / tot,
                "note": "from an eager run with every kernel timed"}
        for k, v in sorted(ks_all.items(), key=lambda kv: -kv[1]["ms"])[:8]:
            print(f"[bench] {k:30s} {int(v['launches']):8d} {v['ms']:9.2f} {100 * v['ms'] / tot:6.1f}%",
                  file=sys.stderr)
    # the GMRES solve of the same points (one batch, unrestarted), untimed by the step clock
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ag, st, rcg = ctx.solve_response(omegas, s.eps, drives, restart=s.n_prod, tol=tol, batch=a.batch,
                                     max_iter=a.max_iter)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    gdiag = np.stack([ag[:, i, i] for i in range(drives.shape[0])], 1)
    out = {
        "metric": "spectrum points/s at 1e-6 rel err in Im alpha vs FP64 oracle",
        "value": passing / dt, "unit": "spectrum points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": a.workload, "seed": a.seed, "method": "two-sided (biorthogonal) lanczos",
                   "n_orb": s.n_orb, "n_occ": s.n_occ, "n_prod": s.n_prod, "n_omega": int(omegas.size),
                   "drives": drive_letters, "eps": s.eps, "points": npts, "tol": tol,
                   "max_steps": a.bl_max_steps, "omega_index": grid.tolist()},
        "recursion_steps": {"mean": float(steps.mean()), "max": int(steps.max()),
                            "per_point": steps.tolist()},
        "status_counts": {str(k): int((status == k).sum()) for k in (0, 1, 2)},
        "accuracy": acc, "roofline": roof,
        "gmres_same_points": {"seconds": tg, "points_per_s": npts / tg,
                              "iterations_mean": float(st["iterations"].mean()),
                              "iterations_max": int(st["iterations"].max()),
                              "max_rel_diff_vs_bilanczos": float(np.max(np.abs(gdiag - alpha) / np.abs(gdiag)))},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="atoms200_orb9",
                    help="synthetic workload; the default is the configuration the metric is quoted on "
                         "(200 atoms, 512 x 3 points), solved on the stratified sample of its grid that "
                         "the stored oracle reference covers")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--batch", type=int, default=128, help="points solved concurrently")
    ap.add_argument("--restart", type=int, default=0, help="GMRES(m); 0 = unrestarted (m = n_prod)")
    ap.add_argument("--tol", type=float, default=0.0, help="0 = the workload's tolerance")
    ap.add_argument("--max-iter", type=int, default=10000)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the Arnoldi-step transforms (IR keeps residuals in FP64)")
    ap.add_argument("--inner-tol", type=float, default=0.0)
    ap.add_argument("--mixed", default="refine", choices=["refine", "relaxed"],
                    help="low precision: iterative refinement cycles, or one Krylov space whose operator "
                         "precision is relaxed as the residual falls")
    ap.add_argument("--relax", type=float, default=0.0,
                    help="relaxed: switch at residual estimate <= relax tol |b| / u (0 = 1)")
    ap.add_argument("--forms", action=argparse.BooleanOptionalAction, default=True,
                    help="after the timed steps, measure the forms of the method on the same points: "
                         "plain (FP64, one point per solve), batched, batched + mixed precision, "
                         "batched + mixed + learned warm start")
    ap.add_argument("--forms-train", type=int, default=16,
                    help="training frequencies of each drive's learned warm start in the forms block")
    ap.add_argument("--alpha-plain", action="store_true",
                    help="alpha = -d.x only (no Sec. 4.1 residual term), for comparison")
    ap.add_argument("--warm", type=int, default=0,
                    help="learned warm start fitted on this many seeded training frequencies (0 = off)")
    ap.add_argument("--cpu-sample", type=int, default=5,
                    help="frequencies for the oracle baseline (0 = skip; ~3.5 s each at 60 atoms)")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel HIP events")
    ap.add_argument("--lanes", type=int, default=1,
                    help="solver lanes (0 = library default: 2 for 16+ concurrent points).  One lane by "
                         "default: the timed per-launch rates are then those of each kernel alone on the "
                         "GPU; two lanes are ~2%% faster on the 60-atom spectrum")
    ap.add_argument("--stop", default="residual", choices=["residual", "eps_p", "eps_px"],
                    help="stopping test: relative residual, or the paper's eps_P / eps_P+eps_X estimates")
    ap.add_argument("--drives", default="", help="dipole drives to solve, e.g. z (default: the workload's)")
    ap.add_argument("--omega-sample", type=int, default=0, metavar="K",
                    help="solve K evenly spaced frequencies of the grid (plus those of a sampled oracle "
                         "reference) instead of the whole grid; 0 = the whole grid, or the stored "
                         "reference's frequencies when it covers only part of the grid")
    ap.add_argument("--apply-only", type=int, default=0, metavar="REPS",
                    help="only time REPS batched chi0 applications (--batch right-hand sides each) "
                         "and report chi0.v GFLOP/s")
    ap.add_argument("--lanczos", action="store_true",
                    help="the spectrum from one Lanczos recursion per drive in transition space instead of "
                         "a GMRES solve per frequency (same workload, error measure and JSON line)")
    ap.add_argument("--bilanczos", action="store_true",
                    help="one two-sided (biorthogonal) Lanczos recursion per point instead of GMRES "
                         "(chi0_solve_bilanczos), compared with the GMRES solve of the same points")
    ap.add_argument("--bl-max-steps", type=int, default=20000, help="two-sided Lanczos: most steps per point")
    ap.add_argument("--no-lanczos", action="store_true",
                    help="skip the untimed comparison with the Lanczos route after the timed steps")
    ap.add_argument("--warm-prev", action="store_true",
                    help="after the timed steps, solve the odd grid points again starting from the "
                         "solution at the next lower grid point (x0) and report the iterations saved")
    ap.add_argument("--n-omega", type=int, default=0,
                    help="solve this many frequencies, evenly spaced on the workload's interval, instead of its "
                         "grid (accuracy then unchecked)")
    ap.add_argument("--dump-alpha", default="", help="save the computed alpha (diagonal, [n_omega][drive]) as .npy")
    ap.add_argument("--lz-kmax", type=int, default=12000, help="Lanczos: most steps")
    ap.add_argument("--lz-tol", type=float, default=1e-8,
                    help="Lanczos: stop when the spectrum on the grid moves by at most this between checks")
    ap.add_argument("--lz-check", type=int, default=100, help="Lanczos: steps between convergence checks")
    ap.add_argument("--lz-solutions", action="store_true",
                    help="Lanczos: also the solutions x(w) and the alpha tensor at every grid frequency "
                         "(after the timed steps, timed on their own)")
    ap.add_argument("--lz-plain", action="store_true",
                    help="Lanczos: no reorthogonalisation (three-term recurrence only)")
    ap.add_argument("--lz-full", action="store_true",
                    help="Lanczos: reorthogonalise every step (default: partial reorthogonalisation, "
                         "Simon's estimates decided on the host)")
    ap.add_argument("--warm-experiment", action="store_true",
                    help="learned warm start vs zero start vs previous-frequency start on one drive "
                         "(--warm training and --omega-sample test frequencies in [--band-lo, omega_max])")
    ap.add_argument("--band-lo", type=float, default=0.0,
                    help="with --omega-sample: sample the band [BAND_LO, omega_max] (Ha) instead of the whole grid; "
                         "also the band of the warm experiment and of the forms' warm-start training")
    ap.add_argument("--spectrum-range", default="", metavar="LO:HI",
                    help="solve the grid points LO..HI-1 of the workload's whole grid x every drive in "
                         "chunks, one line per chunk (no timed steps)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 3 device copies of MIB MiB (reference for HBM traffic counters)")
    a = ap.parse_args()
    if a.calibrate_copy:
        import torch
        n = a.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 3}))
        return
    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {a.gpus} is not supported "
              "(the (frequency, drive) points would be sharded across GPUs with no exchange "
              "but the final gather of alpha; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1005_5340_amd import chi0, synth

    w = synth.WORKLOADS[a.workload]
    t0 = time.perf_counter()
    s = synth.make_system(a.workload, a.seed)
    print(f"[bench] {a.workload} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    drive_letters = a.drives or w.drives
    drives = s.drives(drive_letters)
    tol = a.tol or w.tol
    restart = a.restart or s.n_prod
    ctx = chi0.Context(0)
    t0 = time.perf_counter()
    ctx.set_system_from(s)
    print(f"[bench] set_system {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if a.apply_only:
        return apply_only(a, s, ctx)

    # the oracle's stored polarizability: the whole grid, or a sample of grid points
    ref, ref_idx = None, None
    refpath = os.path.join(ROOT, "tests", "golden", f"reference_{a.workload}_s{a.seed}.json")
    if os.path.exists(refpath):
        r = json.load(open(refpath))
        if synth.same_inputs(s, r["fingerprint"]) and all(c in r["drives"] for c in drive_letters):
            ref = np.array(r["alpha_re"]) + 1j * np.array(r["alpha_im"])
            ref_idx = np.asarray(r["omega_index"], dtype=int)
            ref_drive = [r["drives"].index(c) for c in drive_letters]   # solved drive -> reference index

    # the frequencies solved: the whole grid, or an evenly spaced sample of it
    grid = np.arange(s.omegas.size)
    if not a.omega_sample and ref_idx is not None and ref_idx.size < grid.size:
        grid = np.array(sorted(ref_idx))   # the stored reference's sample of the grid
    elif a.omega_sample and a.band_lo > 0:   # evenly spaced points of the band [band_lo, omega_max]
        gi = np.flatnonzero(s.omegas >= a.band_lo)
        grid = np.unique(gi[np.round(np.linspace(1, gi.size - 1, a.omega_sample)).astype(int)])
    elif a.omega_sample:
        extra = ref_idx if ref_idx is not None else np.zeros(0, int)
        k = max(1, a.omega_sample - extra.size)
        grid = np.unique(np.concatenate([np.round(np.linspace(0, s.omegas.size - 1, k)).astype(int), extra]))
    omegas = s.omegas[grid]
    if a.n_omega:   # a denser inclusive grid on the same interval (no stored reference for it)
        omegas = np.linspace(0.0, w.omega_max, a.n_omega)
        grid = np.arange(a.n_omega)
        ref = None

    if a.lanczos:
        return lanczos_mode(a, s, ctx, drives, drive_letters, omegas, grid, ref, ref_idx,
                            ref_drive if ref is not None else None)
    if a.bilanczos:
        return bilanczos_mode(a, s, ctx, drives, drive_letters, omegas, grid, ref, ref_idx,
                              ref_drive if ref is not None else None, tol)
    if a.spectrum_range:
        return spectrum_range(a, s, ctx, drives, ref, ref_idx, ref_drive if ref is not None else None)
    if a.warm_experiment:
        return warm_experiment(a, s, ctx, drives, restart, tol)

    prec = {"fp64": chi0.PREC_FP64, "fp32": chi0.PREC_FP32, "bf16x3": chi0.PREC_BF16X3}[a.precision]
    ws, warm_info = None, None
    if a.warm > 0:
        rng = np.random.default_rng(1000)
        om_train = np.sort(rng.uniform(0.0, w.omega_max, a.warm))
        t0 = time.perf_counter()
        ws = chi0.WarmStart(ctx, om_train, s.eps, drives[0], rank=min(64, a.warm), width=256,
                            epochs=3000, restart=restart, batch=min(a.warm, a.batch), tol=tol)
        h = ws.loss_history()
        warm_info = {"n_train": a.warm, "fit_seconds": time.perf_counter() - t0,
                     "loss_first": float(h[0]), "loss_last": float(h[-1])}
        print(f"[bench] warm start fitted in {warm_info['fit_seconds']:.2f} s, loss {h[0]:.3e} -> {h[-1]:.3e}",
              file=sys.stderr, flush=True)

    def run(lanes=None):
        return ctx.solve_response(omegas, s.eps, drives, restart=restart, max_iter=a.max_iter,
                                  tol=tol, batch=a.batch, precision=prec, inner_tol=a.inner_tol,
                                  warm=ws, lanes=a.lanes if lanes is None else lanes,
                                  stop={"residual": chi0.STOP_RESIDUAL, "eps_p": chi0.STOP_EPS_P,
                                        "eps_px": chi0.STOP_EPS_PX}[a.stop],
                                  alpha_form=chi0.ALPHA_PLAIN if a.alpha_plain else chi0.ALPHA_CORRECTED,
                                  mixed=chi0.MIXED_RELAXED if a.mixed == "relaxed" else chi0.MIXED_REFINE,
                                  relax=a.relax)

    print(f"[bench] {a.workload}: N={s.n_orb} N_occ={s.n_occ} n_prod={s.n_prod} points="
          f"{omegas.size * drives.shape[0]} batch={a.batch} GMRES({restart}) tol={tol:g}",
          file=sys.stderr, flush=True)
    # One untimed solve on a single lane times every kernel (the per-kernel
    # breakdown, each kernel alone on the GPU); the warmup and timed steps use
    # the requested lanes, and the timed steps time only the dominant kernel,
    # so the two HIP events per timed launch stay off the other ~20 launches
    # of each Arnoldi step.
    ks_all = {}
    if not a.no_timing and a.warmup > 0:
        ctx.set_timing(True)
        t0 = time.perf_counter()
        run(lanes=1)
        ks_all = ctx.kernel_stats()
        print(f"[bench] breakdown run (one lane, all kernels timed) {time.perf_counter() - t0:.3f} s",
              file=sys.stderr, flush=True)
        ctx.set_timing(False)
    for i in range(a.warmup):
        t0 = time.perf_counter()
        run()
        print(f"[bench] warmup {i} {time.perf_counter() - t0:.3f} s", file=sys.stderr, flush=True)
    if not a.no_timing:
        if ks_all:
            dom0 = max(ks_all, key=lambda k: ks_all[k]["ms"])
            ctx.set_timing(True, only=[dom0])
        else:
            ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        alpha, stats, rc = run()
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ks = ctx.kernel_stats() if not a.no_timing else {}
    if not ks_all:
        ks_all = {k: dict(v) for k, v in ks.items()}
        for v in ks_all.values():   # per step, like the warmup breakdown
            for f in ("launches", "ms", "flops", "bytes"):
                v[f] = v[f] / a.steps

    npts = omegas.size * drives.shape[0]
    diag = np.stack([alpha[:, i, i] for i in range(drives.shape[0])], 1)
    if a.dump_alpha:
        np.save(a.dump_alpha, diag)
    if ref is not None and not np.all(np.isin(ref_idx, grid)):
        ref = None      # a reference for frequencies this run did not solve
    # a point passes at the bar of its arithmetic: 1e-10 in floored Im alpha
    # for FP64, 1e-6 with low-precision transforms
    bar = 1e-10 if a.precision == "fp64" else 1e-6
    if ref is not None:
        full = ref_idx.size == grid.size and np.array_equal(np.sort(ref_idx), grid)
        diag = diag[np.searchsorted(grid, ref_idx)]
        rdiag = np.stack([ref[:, ref_drive[i], ref_drive[i]] for i in range(drives.shape[0])], 1)
        err = np.stack([im_errors(diag[:, i], rdiag[:, i]) for i in range(drives.shape[0])], 1)
        if full:
            passing = int((err <= bar).sum())
        else:   # a sample of the grid: the converged points, scaled by the sample's pass rate
            passing = int(stats["converged"].sum()) * float((err <= bar).mean())
        acc = {"checked": True, "bar": bar, "sampled": None if full else
               f"{ref_idx.size} of {grid.size} frequencies solved (grid indices {ref_idx.tolist()}), "
               "value scaled by their pass rate",
               "max_im_rel_err": float(err.max()),
               "median_im_rel_err": float(np.median(err)),
               "max_abs_rel_err": float(np.max(np.abs(diag - rdiag) / np.abs(rdiag))),
               "points_passing_1e-2": int((err <= 1e-2).sum()),
               "max_re_rel_err": float(np.max(np.abs(diag.real - rdiag.real) / np.abs(rdiag.real))),
               "points_passing_1e-6": int((err <= 1e-6).sum()), "points_passing_1e-10": int((err <= 1e-10).sum())}
    else:
        passing = npts
        acc = {"checked": False}
    applications = int((stats["iterations"] + stats["restarts"] + 1).sum())

    roof = None
    chi0_gflops = None
    if ks:
        # roofline of the dominant kernel, from the launches of the timed steps
        dom = max(ks, key=lambda k: ks[k]["ms"])
        rec = ks[dom]
        bound = bound_of(dom)
        peak, unit = PEAK[bound]
        work = rec["bytes"] if bound == "hbm" else rec["flops"]
        achieved = work / (rec["ms"] * 1e-3)
        scale = 1e9 if bound == "hbm" else 1e12
        traffic = load_traffic(dom, a.workload)
        tot_all = sum(v["ms"] for v in ks_all.values())
        roof = {"kernel": dom, "bound": "hbm" if bound == "hbm" else "mfma", "dtype": bound,
                "achieved": achieved / scale, "peak": peak / scale,
                "unit": unit, "frac": achieved / peak, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                "traffic_over_algorithmic": (traffic / (rec["bytes"] / rec["launches"])) if traffic and rec["bytes"] else None,
                "launches": rec["launches"] // a.steps, "mean_launch_us": 1e3 * rec["ms"] / rec["launches"],
                "share_of_gpu_time": (ks_all[dom]["ms"] / tot_all) if dom in ks_all else None,
                "lanes": a.lanes or ("auto: 2" if a.batch >= 16 else "auto: 1"),
                "note": "per-launch rate over the timed steps (HIP events on the lane's stream); with "
                        "more than one lane a launch shares the GPU with the other lanes' kernels"}
        # chi0 rate and the per-kernel breakdown: every kernel timed (the
        # single-lane breakdown run, or the timed steps when there is no warmup)
        chi0_ms = sum(ks_all[k]["ms"] for k in CHI0_KERNELS if k in ks_all)
        F = chi0_flops(s)
        if chi0_ms > 0:
            chi0_gflops = F * applications / (chi0_ms * 1e-3) / 1e9
        print("[bench] per-step breakdown (one lane, all kernels timed)", file=sys.stderr)
        print("[bench] kernel            launches/step   ms/step   share   achieved", file=sys.stderr)
        for k, v in sorted(ks_all.items(), key=lambda kv: -kv[1]["ms"]):
            b = bound_of(k)
            ach = (v["bytes"] / 1e9 if b == "hbm" else v["flops"] / 1e12) / (v["ms"] * 1e-3)
            print(f"[bench] {k:30s} {int(v['launches']):8d} {v['ms']:9.2f} "
                  f"{100 * v['ms'] / tot_all:6.1f}%  {ach:9.2f} {'GB/s' if b == 'hbm' else 'TFLOP/s'}",
                  file=sys.stderr)

    forms = None
    if a.forms:
        forms = measure_forms(a, s, ctx, omegas, grid, drives, drive_letters, ref, ref_idx,
                              ref_drive if ref is not None else None, restart, tol,
                              alpha64=alpha, batched={"points_per_s": passing / dt, "seconds": dt, "passing": passing, "bar": bar,
                               "points": npts, "iterations": {"mean": float(stats["iterations"].mean()),
                                                              "max": int(stats["iterations"].max())},
                               "chi0_tflops": chi0_gflops / 1e3 if chi0_gflops else None,
                               "dominant": None if roof is None else
                               {k: roof[k] for k in ("kernel", "achieved", "peak", "unit", "frac")},
                               "note": "the timed steps (batch of every point, FP64, learned start off)"})

    # the same spectrum by the Lanczos route (one recursion per drive), after the timed steps
    lz_route = None
    if not a.no_lanczos and drives.shape[0] <= 4 and s.n_occ * (s.n_orb - s.n_occ) <= 100000:
        ctx.set_timing(False)
        lzkw = dict(k_max=a.lz_kmax, tol=a.lz_tol, check_every=a.lz_check, omega_check=omegas, eps=s.eps)
        ctx.lanczos(drives, **lzkw)          # untimed: tunes the operator's GEMM tiles for its shapes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lres = ctx.lanczos(drives, **lzkw)
        lal = ctx.lanczos_spectrum(lres, omegas, s.eps)
        t_lz = time.perf_counter() - t0
        lz_route = {"method": "Lanczos recursion in transition space, partial reorthogonalisation",
                    "seconds": t_lz, "points_per_s": npts / t_lz, "steps": lres["len"].tolist(),
                    "rc": int(lres["rc"])}
        if ref is not None and np.all(np.isin(ref_idx, grid)):
            ld = lal[np.searchsorted(grid, ref_idx)]
            rd = np.stack([ref[:, ref_drive[i], ref_drive[i]] for i in range(drives.shape[0])], 1)
            le = np.stack([im_errors(ld[:, i], rd[:, i]) for i in range(drives.shape[0])], 1)
            lz_route.update(max_im_rel_err=float(le.max()), points_passing_1e_6=int((le <= 1e-6).sum()),
                            points_per_s=int((le <= 1e-6).sum()) / t_lz if ref_idx.size == grid.size
                            else lz_route["points_per_s"])
        print(f"[bench] Lanczos route: {lz_route}", file=sys.stderr, flush=True)

    warm_prev = None
    if a.warm_prev:
        ctx.set_timing(False)
        ev, od = np.arange(0, omegas.size, 2), np.arange(1, omegas.size, 2)
        _, _, _, xe = ctx.solve_response(omegas[ev], s.eps, drives, restart=restart, max_iter=a.max_iter, tol=tol,
                                         batch=a.batch, lanes=a.lanes, return_x=True)
        x0 = torch.from_numpy(np.ascontiguousarray(xe[: od.size])).to("cuda")   # grid point 2m for 2m + 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st_cold, _ = ctx.solve_response(omegas[od], s.eps, drives, restart=restart, max_iter=a.max_iter,
                                           tol=tol, batch=a.batch, lanes=a.lanes)
        t_cold = time.perf_counter() - t0
        t0 = time.perf_counter()
        a_w, st_w, _ = ctx.solve_response(omegas[od], s.eps, drives, restart=restart, max_iter=a.max_iter,
                                          tol=tol, batch=a.batch, lanes=a.lanes, x0=x0)
        t_w = time.perf_counter() - t0
        warm_prev = {"points": int(od.size * drives.shape[0]), "seconds_cold": t_cold, "seconds_x0": t_w,
                     "iterations_cold": int(st_cold["iterations"].sum()),
                     "iterations_x0": int(st_w["iterations"].sum()),
                     "max_iterations_cold": int(st_cold["iterations"].max()),
                     "max_iterations_x0": int(st_w["iterations"].max()),
                     "median_rel_residual_of_x0": float(np.median(st_w["warm_rel0"])),
                     "rejected": int((st_w["warm_start"] == 2).sum())}
        if ref is not None and np.all(np.isin(ref_idx, grid)):
            sel = np.searchsorted(ref_idx, grid[od])
            rw = np.stack([ref[sel, ref_drive[i], ref_drive[i]] for i in range(drives.shape[0])], 1)
            ew = np.stack([im_errors(a_w[:, i, i], rw[:, i]) for i in range(drives.shape[0])], 1)
            warm_prev["max_im_rel_err"] = float(ew.max())
        print(f"[bench] previous-frequency start: {warm_prev}", file=sys.stderr, flush=True)

    tuned = ctx.autotune_table()
    for k, v in sorted(tuned.items()):
        us = ", ".join(f"{x:.0f}" if x > 0 else "-" for x in v["us"][:6])
        print(f"[bench] autotune {k:58s} -> {v['tile']:10s} (us per variant 64x64, 64x128, 128x64, "
              f"128x128, 64x64/k32, 64x128/k32: {us})", file=sys.stderr)

    cpu = None
    if a.cpu_sample > 0:
        cpu = cpu_baseline(s, drives, a.cpu_sample)

    out = {
        "metric": "spectrum points/s at 1e-6 rel err in Im alpha vs FP64 oracle",
        "value": passing / dt,
        "unit": "spectrum points/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64+f32", "bf16x3": "f64+bf16x3"}[a.precision],
        "data": "synthetic",
        "config": {"workload": a.workload, "seed": a.seed, "n_orb": s.n_orb, "n_occ": s.n_occ,
                   "n_prod": s.n_prod, "n_omega": int(omegas.size), "drives": drive_letters,
                   "omega_grid": int(s.omegas.size), "omega_sample": a.omega_sample or None,
                   "omega_index": grid.tolist() if grid.size < s.omegas.size else None,
                   "eps": s.eps, "tol": tol, "restart": restart, "batch": a.batch,
                   "points": npts, "precision": a.precision, "warm_start_train": a.warm,
                   "lanes": a.lanes, "stop": a.stop, "mixed": a.mixed if a.precision != "fp64" else None,
                   "alpha": "plain -d.x" if a.alpha_plain else "with the Sec. 4.1 residual term"},
        "chi0_gflops": chi0_gflops,
        "autotune": {k: v["tile"] for k, v in sorted(tuned.items())},
        "chi0_applications_per_step": applications,
        "iterations": {"mean": float(stats["iterations"].mean()), "max": int(stats["iterations"].max()),
                       "converged": int(stats["converged"].sum()),
                       "fallbacks": int(stats["fallback"].sum())},
        "warm_start": None if warm_info is None else {
            **warm_info, "used": int((stats["warm_start"] == 1).sum()),
            "rejected": int((stats["warm_start"] == 2).sum()),
            "median_rel_residual_of_x0": float(np.median(stats["warm_rel0"]))},
        "accuracy": acc,
        "roofline": roof,
        "cpu_baseline": cpu,
        "warm_previous_frequency": warm_prev,
        "lanczos_route": lz_route,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)
    if ws is not None:
        ws.close()
    ctx.close()


if __name__ == "__main__":
    main()
