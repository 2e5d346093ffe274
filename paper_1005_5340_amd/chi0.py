"""Python binding of libchi0 (argument marshalling only).

Every computation runs inside the HIP library; this module converts NumPy
arrays and PyTorch device tensors into the pointers of the C-ABI declared in
include/chi0.h and turns return codes into exceptions.  It loads the in-tree
`libchi0.so` and raises if it is missing: there is no fallback.

Names follow the C-ABI: `Context.set_system`, `Context.apply`,
`Context.solve_response` (chi0_set_system, chi0_apply, chi0_solve_response).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

__all__ = ["Chi0Error", "Context", "WarmStart", "lib", "LIB_PATH", "PREC_FP64", "PREC_FP32",
           "PREC_BF16X3", "SolveStats", "NOT_CONVERGED", "debug_eigh", "STOP_RESIDUAL", "STOP_EPS_P",
           "STOP_EPS_PX", "ALPHA_CORRECTED", "ALPHA_PLAIN", "MIXED_REFINE", "MIXED_RELAXED", "LanczosOpts", "LZ_REORTH_NONE", "LZ_REORTH_FULL", "LZ_REORTH_FULL2", "LZ_REORTH_PARTIAL", "lanczos_poles"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchi0.so")
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2
ORTHO_AUTO, ORTHO_CGS2, ORTHO_DCGS2 = 0, 1, 2
STOP_RESIDUAL, STOP_EPS_P, STOP_EPS_PX = 0, 1, 2
ALPHA_CORRECTED, ALPHA_PLAIN = 0, 1
MIXED_REFINE, MIXED_RELAXED = 0, 1
LZ_REORTH_NONE, LZ_REORTH_FULL, LZ_REORTH_FULL2, LZ_REORTH_PARTIAL = 0, 1, 2, 3
NOT_CONVERGED = 1
_ERRORS = {-1: "EINVAL", -2: "ENOSYS", -3: "ENOMEM", -4: "EHIP", -5: "ENONFINITE", -6: "EASYM"}

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("precision", C.c_int32), ("batch", C.c_int32), ("inner_tol", C.c_double),
                ("warm", C.c_void_p), ("ortho", C.c_int32), ("lanes", C.c_int32),
                ("stop", C.c_int32), ("alpha_form", C.c_int32), ("x0", C.c_void_p),
                ("warm_drive", C.POINTER(C.c_void_p)), ("mixed", C.c_int32), ("relax", C.c_double)]


class WsCfg(C.Structure):
    _fields_ = [("rank", C.c_int32), ("width", C.c_int32), ("n_freq", C.c_int32),
                ("epochs", C.c_int32), ("w_scale", C.c_double), ("lr", C.c_double),
                ("seed", C.c_uint64), ("restart", C.c_int32), ("batch", C.c_int32),
                ("tol", C.c_double), ("reserved", C.c_int32 * 4)]


class PointStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("breakdown", C.c_int32), ("fallback", C.c_int32), ("warm_start", C.c_int32),
                ("rel_residual", C.c_double), ("warm_rel0", C.c_double),
                ("eps_x", C.c_double), ("eps_p", C.c_double), ("low_prec_steps", C.c_int32),
                ("reserved", C.c_int32)]


class LanczosOpts(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("reorth", C.c_int32), ("tol", C.c_double),
                ("check_every", C.c_int32), ("n_check", C.c_int32), ("omega_check", _dp),
                ("eps", C.c_double), ("graph", C.c_int32), ("n_x", C.c_int32), ("omega_x", _dp),
                ("x", _dp), ("alpha_x", _dp), ("reserved", C.c_int32 * 2)]


class TuneRecord(C.Structure):
    _fields_ = [("key", C.c_char * 96), ("tile", C.c_char * 16), ("variant", C.c_int32),
                ("us", C.c_float * 8)]


class KernelRecord(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


SolveStats = np.dtype([("iterations", np.int32), ("restarts", np.int32), ("converged", np.int32),
                       ("breakdown", np.int32), ("fallback", np.int32), ("warm_start", np.int32),
                       ("rel_residual", np.float64), ("warm_rel0", np.float64),
                       ("eps_x", np.float64), ("eps_p", np.float64), ("low_prec_steps", np.int32)])

_LIB = None


def lib():
    """Load libchi0.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # PyTorch wheels ship their own libamdhip64.so.7.  Loading torch first makes
    # the dynamic linker resolve this library's HIP runtime to the same copy,
    # so one runtime owns the GPU and torch tensors can be passed to chi0_apply.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    L.chi0_create.argtypes = [C.POINTER(C.c_void_p), C.c_int]
    L.chi0_create.restype = C.c_int
    L.chi0_destroy.argtypes = [C.c_void_p]
    L.chi0_destroy.restype = None
    L.chi0_last_error.argtypes = [C.c_void_p]
    L.chi0_last_error.restype = C.c_char_p
    L.chi0_set_system.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_int32, C.c_int32, C.c_double,
                                  _dp, _dp, _i32p, C.c_int32, _i32p, _i64p, _dp, _dp]
    L.chi0_set_system.restype = C.c_int
    L.chi0_get_sizes.argtypes = [C.c_void_p, _i32p, _i32p, _i32p, _i32p]
    L.chi0_get_sizes.restype = C.c_int
    L.chi0_apply.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_double, C.c_void_p, C.c_void_p,
                             C.c_int32, C.c_void_p]
    L.chi0_apply.restype = C.c_int
    L.chi0_apply_noalloc.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
    L.chi0_apply_noalloc.restype = C.c_int
    L.chi0_solve_opts_default.argtypes = [C.POINTER(SolveOpts)]
    L.chi0_solve_opts_default.restype = None
    L.chi0_solve_response.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_double, C.c_int32, _dp,
                                      C.POINTER(SolveOpts), _dp, C.POINTER(PointStats)]
    L.chi0_solve_response.restype = C.c_int
    L.chi0_solve_response_x.argtypes = list(L.chi0_solve_response.argtypes) + [_dp]
    L.chi0_solve_response_x.restype = C.c_int
    L.chi0_set_timing.argtypes = [C.c_void_p, C.c_int32]
    L.chi0_set_timing.restype = C.c_int
    L.chi0_set_autotune.argtypes = [C.c_void_p, C.c_int32]
    L.chi0_set_autotune.restype = C.c_int
    L.chi0_set_graphs.argtypes = [C.c_void_p, C.c_int32]
    L.chi0_set_graphs.restype = C.c_int
    L.chi0_autotune_table.argtypes = [C.c_void_p, C.POINTER(TuneRecord), C.c_int32]
    L.chi0_autotune_table.restype = C.c_int
    L.chi0_set_timing_filter.argtypes = [C.c_void_p, C.c_char_p]
    L.chi0_set_timing_filter.restype = C.c_int
    L.chi0_kernel_stats.argtypes = [C.c_void_p, C.POINTER(KernelRecord), C.c_int32]
    L.chi0_kernel_stats.restype = C.c_int
    L.chi0_ws_cfg_default.argtypes = [C.POINTER(WsCfg)]
    L.chi0_ws_cfg_default.restype = None
    L.chi0_ws_fit.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_double, _dp, C.POINTER(WsCfg),
                              C.POINTER(C.c_void_p)]
    L.chi0_ws_fit.restype = C.c_int
    L.chi0_ws_free.argtypes = [C.c_void_p]
    L.chi0_ws_free.restype = None
    L.chi0_ws_predict.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_void_p]
    L.chi0_ws_predict.restype = C.c_int
    L.chi0_ws_loss_history.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int32]
    L.chi0_ws_loss_history.restype = C.c_int
    L.chi0_ws_debug_dims.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.chi0_ws_debug_dims.restype = C.c_int
    L.chi0_ws_debug_params.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64, C.c_int32]
    L.chi0_ws_debug_params.restype = C.c_int
    L.chi0_ws_debug_loss_grad.argtypes = [C.c_void_p, C.c_int32, _dp, C.POINTER(C.c_float),
                                          C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.chi0_ws_debug_loss_grad.restype = C.c_int
    L.chi0_debug_lz_passes.argtypes = [C.c_void_p, _i32p, _dp, C.c_int32]
    L.chi0_debug_lz_passes.restype = C.c_int
    L.chi0_debug_eigh.argtypes = [C.c_int32, _dp, _dp, _dp]
    L.chi0_debug_eigh.restype = C.c_int
    L.chi0_lanczos_opts_default.argtypes = [C.POINTER(LanczosOpts)]
    L.chi0_lanczos_opts_default.restype = None
    L.chi0_lanczos.argtypes = [C.c_void_p, C.c_int32, _dp, C.POINTER(LanczosOpts), _dp, _dp, _dp, _i32p]
    L.chi0_lanczos.restype = C.c_int
    L.chi0_lanczos_spectrum.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, _dp, _i32p, C.c_int32,
                                        _dp, C.c_double, _dp]
    L.chi0_lanczos_spectrum.restype = C.c_int
    L.chi0_lanczos_poles.argtypes = [C.c_int32, _dp, _dp, C.c_double, _dp, _dp]
    L.chi0_lanczos_poles.restype = C.c_int
    L.chi0_solve_bilanczos.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_double, C.c_int32, _dp, C.c_double,
                                       C.c_int32, _dp, _i32p, _i32p]
    L.chi0_solve_bilanczos.restype = C.c_int
    _LIB = L
    return L


class Chi0Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chi0 error {code} ({_ERRORS.get(code, '?')}): {msg}")
        self.code = code


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape}, got {a.shape}")
    return a


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class Context:
    """One chi0 context bound to a HIP device (device=-1: host-only validation)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.chi0_create(C.byref(h), int(device))
        if rc != 0:
            raise Chi0Error(rc, self._L.chi0_last_error(None).decode())
        self._h = h
        self.device = device

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None):
            self._L.chi0_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int, allow_warning: bool = False) -> int:
        if rc < 0 or (rc > 0 and not allow_warning):
            raise Chi0Error(rc, self._L.chi0_last_error(self._h).decode())
        return rc

    @property
    def last_error(self) -> str:
        return self._L.chi0_last_error(self._h).decode()

    # ---------------------------------------------------------------- system
    def set_system(self, n_atoms, positions, n_orb, n_occ, occ_factor, eigenvalues, X,
                   atom_orb_offset, n_prod, prod_atoms, vblock_offset, vblock, K):
        """chi0_set_system; host arrays are copied."""
        pos = None if positions is None else _f64(positions, (n_atoms, 3))
        eig = _f64(eigenvalues, (n_orb,))
        Xa = _f64(X, (n_orb, n_orb))
        aoff = np.ascontiguousarray(atom_orb_offset, dtype=np.int32)
        pat = np.ascontiguousarray(prod_atoms, dtype=np.int32)
        voff = np.ascontiguousarray(vblock_offset, dtype=np.int64)
        vb = _f64(vblock)
        Ka = _f64(K, (n_prod, n_prod))
        if aoff.size != n_atoms + 1 or pat.size != 2 * n_prod or voff.size != n_prod + 1:
            raise ValueError("inconsistent array sizes")
        self._keep = (pos, eig, Xa, aoff, pat, voff, vb, Ka)
        rc = self._L.chi0_set_system(self._h, int(n_atoms), _ptr(pos), int(n_orb), int(n_occ),
                                     float(occ_factor), _ptr(eig), _ptr(Xa), _ptr(aoff, _i32p),
                                     int(n_prod), _ptr(pat, _i32p), _ptr(voff, _i64p), _ptr(vb),
                                     _ptr(Ka))
        self._keep = None
        self._check(rc)

    def set_system_from(self, sys):
        """Convenience: pass a `synth.System` (or anything with the same fields)."""
        self.set_system(sys.n_atoms, sys.positions, sys.n_orb, sys.n_occ, sys.occ_factor,
                        sys.eigenvalues, sys.X, sys.atom_orb_offset, sys.n_prod, sys.prod_atoms,
                        sys.vblock_offset, sys.vblock, sys.K)

    def sizes(self):
        v = [C.c_int32() for _ in range(4)]
        self._check(self._L.chi0_get_sizes(self._h, *[C.byref(x) for x in v]))
        return dict(n_orb=v[0].value, n_occ=v[1].value, n_prod=v[2].value, n_atoms=v[3].value)

    # ----------------------------------------------------------------- apply
    def apply(self, omega, eps: float, z, out=None, precision: int = PREC_FP64, stream=None):
        """out[r] = chi0(omega[r]) z[r] for torch complex128 CUDA tensors z [n_rhs, n_prod].

        Enqueued on `stream` (default: torch's current stream); returns `out`.
        """
        import torch
        om = _f64(np.atleast_1d(omega))
        if not (z.is_cuda and z.dtype == torch.complex128 and z.is_contiguous() and z.dim() == 2):
            raise ValueError("z must be a contiguous complex128 CUDA tensor [n_rhs, n_prod]")
        if z.shape[0] != om.size:
            raise ValueError("one frequency per row of z")
        if out is None:
            out = torch.empty_like(z)
        if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()
                and out.shape == z.shape):
            raise ValueError("out must match z")
        if stream is None:
            stream = torch.cuda.current_stream(z.device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        rc = self._L.chi0_apply(self._h, int(om.size), _ptr(om), float(eps),
                                C.c_void_p(z.data_ptr()), C.c_void_p(out.data_ptr()),
                                int(precision), C.c_void_p(handle))
        self._check(rc)
        return out

    # ---------------------------------------------------------------- solve
    def apply_noalloc(self, omega, eps: float, z, out=None, stream=None):
        """chi0_apply_noalloc: FP64 out[r] = chi0(omega[r]) z[r] with the library's static
        device scratch (the call allocates nothing; the GPU's scratch is shared by every
        call, so calls must not overlap).  Same arguments as `apply` without precision."""
        import torch
        om = _f64(np.atleast_1d(omega))
        if not (z.is_cuda and z.dtype == torch.complex128 and z.is_contiguous() and z.dim() == 2):
            raise ValueError("z must be a contiguous complex128 CUDA tensor [n_rhs, n_prod]")
        if z.shape[0] != om.size:
            raise ValueError("one frequency per row of z")
        if out is None:
            out = torch.empty_like(z)
        if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()
                and out.shape == z.shape):
            raise ValueError("out must match z")
        if stream is None:
            stream = torch.cuda.current_stream(z.device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        rc = self._L.chi0_apply_noalloc(self._h, int(om.size), _ptr(om), float(eps),
                                        C.c_void_p(z.data_ptr()), C.c_void_p(out.data_ptr()),
                                        C.c_void_p(handle))
        self._check(rc)
        return out

    def solve_bilanczos(self, omega, eps: float, V_ext, tol: float = 1e-10, max_steps: int = 20000):
        """Two-sided Lanczos polarizability (chi0_solve_bilanczos).

        Returns (alpha [n_omega, n_drive] complex (alpha_ii), steps [n_omega, n_drive],
        status [n_omega, n_drive] (0 converged, 1 max_steps, 2 breakdown), rc) where rc is
        0 or NOT_CONVERGED.
        """
        om = _f64(np.atleast_1d(omega))
        D = _f64(np.atleast_2d(V_ext))
        nd = D.shape[0]
        alpha = np.zeros((om.size, nd, 2))
        steps = np.zeros((om.size, nd), np.int32)
        status = np.zeros((om.size, nd), np.int32)
        rc = self._L.chi0_solve_bilanczos(self._h, int(om.size), _ptr(om), float(eps), int(nd), _ptr(D),
                                          float(tol), int(max_steps), _ptr(alpha), _ptr(steps, _i32p),
                                          _ptr(status, _i32p))
        self._check(rc, allow_warning=True)
        return alpha[..., 0] + 1j * alpha[..., 1], steps, status, rc

    def solve_response(self, omega, eps: float, V_ext, restart: int = 30, max_iter: int = 10000,
                       tol: float = 1e-10, batch: int = 1, precision: int = PREC_FP64,
                       inner_tol: float = 0.0, warm: "WarmStart" = None, ortho: int = ORTHO_AUTO,
                       return_x: bool = False, lanes: int = 0, stop: int = STOP_RESIDUAL, x0=None,
                       alpha_form: int = ALPHA_CORRECTED, mixed: int = MIXED_REFINE, relax: float = 0.0):
        """GMRES polarizability over a frequency grid.

        Returns (alpha [n_omega, n_drive, n_drive] complex, stats [n_omega, n_drive], rc)
        where rc is 0 or NOT_CONVERGED; with return_x also the solutions
        x [n_omega, n_drive, n_prod] complex (chi0_solve_response_x).  x0: optional start
        vectors, a contiguous complex128 device tensor [n_omega, n_drive, n_prod].  warm: a
        WarmStart for every drive, or a list with one WarmStart (or None) per drive.
        """
        om = _f64(np.atleast_1d(omega))
        D = _f64(np.atleast_2d(V_ext))
        nd = D.shape[0]
        o = SolveOpts()
        self._L.chi0_solve_opts_default(C.byref(o))
        o.restart, o.max_iter, o.tol = int(restart), int(max_iter), float(tol)
        o.batch, o.precision, o.inner_tol = int(batch), int(precision), float(inner_tol)
        if isinstance(warm, (list, tuple)):     # one warm start per drive (None: zero start)
            if len(warm) != nd:
                raise ValueError("one warm start (or None) per drive")
            wd = (C.c_void_p * nd)(*[w._h if w is not None else None for w in warm])
            o.warm_drive = C.cast(wd, C.POINTER(C.c_void_p))
        else:
            o.warm = warm._h if warm is not None else None
        o.ortho = int(ortho)
        o.lanes = int(lanes)
        o.stop = int(stop)
        o.alpha_form = int(alpha_form)
        o.mixed, o.relax = int(mixed), float(relax)
        if x0 is not None:
            import torch
            n_prod = self.sizes()["n_prod"]
            if (not isinstance(x0, torch.Tensor) or x0.device.type != "cuda" or x0.dtype != torch.complex128
                    or not x0.is_contiguous() or tuple(x0.shape) != (om.size, nd, n_prod)):
                raise ValueError("x0 must be a contiguous complex128 cuda tensor [n_omega, n_drive, n_prod]")
            o.x0 = x0.data_ptr()
        alpha = np.zeros((om.size, nd, nd, 2))
        st = (PointStats * max(1, om.size * nd))()
        if return_x:
            n_prod = self.sizes()["n_prod"]
            x = np.zeros((om.size, nd, n_prod, 2))
            rc = self._L.chi0_solve_response_x(self._h, int(om.size), _ptr(om), float(eps), int(nd),
                                               _ptr(D), C.byref(o), _ptr(alpha), st, _ptr(x))
        else:
            rc = self._L.chi0_solve_response(self._h, int(om.size), _ptr(om), float(eps), int(nd),
                                             _ptr(D), C.byref(o), _ptr(alpha), st)
        self._check(rc, allow_warning=True)
        stats = np.zeros((om.size, nd), dtype=SolveStats)
        flat = stats.reshape(-1)
        for i in range(om.size * nd):
            flat[i] = (st[i].iterations, st[i].restarts, st[i].converged, st[i].breakdown,
                       st[i].fallback, st[i].warm_start, st[i].rel_residual, st[i].warm_rel0,
                       st[i].eps_x, st[i].eps_p, st[i].low_prec_steps)
        a = alpha[..., 0] + 1j * alpha[..., 1]
        if return_x:
            return a, stats, rc, x[..., 0] + 1j * x[..., 1]
        return a, stats, rc

    def lanczos(self, drives, k_max: int = 4000, reorth: int = LZ_REORTH_PARTIAL, tol: float = 0.0,
                check_every: int = 100, omega_check=None, eps: float = 0.0, graph: bool = False,
                omega_x=None) -> dict:
        """Lanczos recursion in transition space for 1..4 drives [n_drive][n_prod] (chi0_lanczos).

        Returns dict(a, b: [n_drive][k_max], c_norm2: [n_drive], len: [n_drive], rc); with
        omega_x also x [n_x][n_drive][n_prod] and alpha_x [n_x][n_drive][n_drive] complex."""
        d = _f64(drives)
        d = d.reshape(-1, d.shape[-1])
        nd = d.shape[0]
        om = None if omega_check is None else _f64(omega_check).ravel()
        omx = None if omega_x is None else _f64(omega_x).ravel()
        o = LanczosOpts()
        self._L.chi0_lanczos_opts_default(C.byref(o))
        o.k_max, o.reorth, o.tol, o.check_every = int(k_max), int(reorth), float(tol), int(check_every)
        o.n_check = 0 if om is None else int(om.size)
        o.omega_check = _ptr(om)
        o.eps, o.graph = float(eps), int(bool(graph))
        x = ax = None
        if omx is not None:
            x = np.zeros((omx.size, nd, d.shape[-1], 2))
            ax = np.zeros((omx.size, nd, nd, 2))
            o.n_x, o.omega_x, o.x, o.alpha_x = int(omx.size), _ptr(omx), _ptr(x), _ptr(ax)
        a = np.zeros((nd, max(int(k_max), 1)))
        b = np.zeros_like(a)
        cn2 = np.zeros(nd)
        ln = np.zeros(nd, np.int32)
        rc = self._check(self._L.chi0_lanczos(self._h, nd, _ptr(d), C.byref(o), _ptr(a), _ptr(b), _ptr(cn2),
                                              _ptr(ln, _i32p)), allow_warning=True)
        out = dict(a=a, b=b, c_norm2=cn2, len=ln, rc=rc)
        if omx is not None:
            out["x"] = x[..., 0] + 1j * x[..., 1]
            out["alpha_x"] = ax[..., 0] + 1j * ax[..., 1]
        return out

    def lanczos_spectrum(self, res: dict, omega, eps: float) -> np.ndarray:
        """alpha_k(omega) [n_omega][n_drive] complex from a lanczos() result (chi0_lanczos_spectrum)."""
        a, b = _f64(res["a"]), _f64(res["b"])
        nd, ld = a.shape
        cn2 = _f64(res["c_norm2"])
        ln = np.ascontiguousarray(res["len"], np.int32)
        om = _f64(omega).ravel()
        out = np.zeros((om.size, nd, 2))
        self._check(self._L.chi0_lanczos_spectrum(self._h, nd, ld, _ptr(a), _ptr(b), _ptr(cn2), _ptr(ln, _i32p),
                                                  int(om.size), _ptr(om), float(eps), _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def debug_lz_passes(self, n_drive: int):
        """Test hook: per step of the last timed partial-reorthogonalisation recursion,
        whether the pass ran and the pre-pass b_j of each drive ([steps], [steps, n_drive])."""
        n = self._L.chi0_debug_lz_passes(self._h, None, None, 0)
        p = np.zeros(max(n, 1), np.int32)
        b = np.zeros((max(n, 1), n_drive))
        self._L.chi0_debug_lz_passes(self._h, _ptr(p, _i32p), _ptr(b), n)
        return p[:n], b[:n]

    def set_graphs(self, enable: bool):
        """Replay repeated chi0_apply calls from a HIP graph (chi0_set_graphs)."""
        self._check(self._L.chi0_set_graphs(self._h, int(bool(enable))))

    # --------------------------------------------------------------- tracing
    def set_timing(self, enable: bool, only=None):
        """Enable per-kernel HIP-event timing; `only` restricts it to the named kernels."""
        names = ",".join(only).encode() if only else None
        self._check(self._L.chi0_set_timing_filter(self._h, names))
        self._check(self._L.chi0_set_timing(self._h, 1 if enable else 0))

    def set_autotune(self, enable: bool, force_variant: int = -1):
        """Tile autotuning on/off; force_variant >= 0 forces that tile variant (tests)."""
        mode = 100 + force_variant if force_variant >= 0 else (1 if enable else 0)
        self._check(self._L.chi0_set_autotune(self._h, mode))

    def autotune_table(self) -> dict:
        """{shape class: dict(tile, variant, us=[per-variant microseconds, 0 = not valid])}."""
        n = self._L.chi0_autotune_table(self._h, None, 0)
        self._check(min(n, 0))
        recs = (TuneRecord * max(1, n))()
        n = self._L.chi0_autotune_table(self._h, recs, n)
        return {recs[i].key.decode(): dict(tile=recs[i].tile.decode(), variant=int(recs[i].variant),
                                           us=[float(x) for x in recs[i].us])
                for i in range(n)}

    def kernel_stats(self) -> dict:
        """{kernel: dict(launches, ms, flops, bytes)} accumulated since set_timing(True)."""
        n = self._L.chi0_kernel_stats(self._h, None, 0)
        self._check(min(n, 0))
        recs = (KernelRecord * max(1, n))()
        n = self._L.chi0_kernel_stats(self._h, recs, n)
        return {recs[i].name.decode(): dict(launches=int(recs[i].launches), ms=float(recs[i].total_ms),
                                            flops=float(recs[i].flops), bytes=float(recs[i].bytes))
                for i in range(n)}


class WarmStart:
    """Learned GMRES warm start (chi0_ws_fit): x0(omega) = U c(omega)."""

    def __init__(self, ctx: Context, omega_train, eps: float, drive, rank: int = 64,
                 width: int = 256, n_freq: int = 16, epochs: int = 3000, lr: float = 2e-3,
                 seed: int = 1234, restart: int = 0, batch: int = 64, tol: float = 1e-10,
                 w_scale: float = 0.0):
        self._L = ctx._L
        self.ctx = ctx
        om = _f64(np.atleast_1d(omega_train))
        d = _f64(drive)
        cfg = WsCfg()
        self._L.chi0_ws_cfg_default(C.byref(cfg))
        cfg.rank, cfg.width, cfg.n_freq, cfg.epochs = int(rank), int(width), int(n_freq), int(epochs)
        cfg.lr, cfg.seed, cfg.restart, cfg.batch = float(lr), int(seed), int(restart), int(batch)
        cfg.tol, cfg.w_scale = float(tol), float(w_scale)
        h = C.c_void_p()
        rc = self._L.chi0_ws_fit(ctx._h, int(om.size), _ptr(om), float(eps), _ptr(d), C.byref(cfg),
                                 C.byref(h))
        ctx._check(rc, allow_warning=True)
        self._h = h
        self.fit_rc = rc

    def close(self):
        if getattr(self, "_h", None):
            self._L.chi0_ws_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def predict(self, omega):
        """x0 for each frequency as a torch complex128 CUDA tensor [n, n_prod]."""
        import torch
        om = _f64(np.atleast_1d(omega))
        n_prod = self.ctx.sizes()["n_prod"]
        out = torch.zeros((om.size, n_prod), dtype=torch.complex128, device="cuda")
        self.ctx._check(self._L.chi0_ws_predict(self._h, int(om.size), _ptr(om), C.c_void_p(out.data_ptr())))
        return out

    def loss_history(self) -> np.ndarray:
        n = self._L.chi0_ws_loss_history(self._h, None, 0)
        buf = np.zeros(max(n, 1), np.float32)
        self._L.chi0_ws_loss_history(self._h, buf.ctypes.data_as(C.POINTER(C.c_float)), n)
        return buf[:n]

    # ------------------------------------------------------------ test hooks
    def dims(self) -> dict:
        d = (C.c_int64 * 7)()
        ws = C.c_double()
        self.ctx._check(self._L.chi0_ws_debug_dims(self._h, d, C.byref(ws)))
        return dict(r=d[0], F=d[1], W=d[2], O=d[3], n_params=d[4], n_freq=d[5], w_scale=ws.value)

    def params(self, new=None) -> np.ndarray:
        n = self.dims()["n_params"]
        if new is not None:
            buf = np.ascontiguousarray(new, dtype=np.float32)
            assert buf.size == n
            self.ctx._check(self._L.chi0_ws_debug_params(self._h, buf.ctypes.data_as(C.POINTER(C.c_float)), n, 1))
            return buf
        buf = np.zeros(n, np.float32)
        self.ctx._check(self._L.chi0_ws_debug_params(self._h, buf.ctypes.data_as(C.POINTER(C.c_float)), n, 0))
        return buf

    def loss_grad(self, omega, target):
        om = _f64(np.atleast_1d(omega))
        tg = np.ascontiguousarray(target, dtype=np.float32)
        n = self.dims()["n_params"]
        loss = np.zeros(1, np.float32)
        g = np.zeros(n, np.float32)
        fp = C.POINTER(C.c_float)
        self.ctx._check(self._L.chi0_ws_debug_loss_grad(self._h, int(om.size), _ptr(om), tg.ctypes.data_as(fp),
                                                        loss.ctypes.data_as(fp), g.ctypes.data_as(fp)))
        return float(loss[0]), g


def lanczos_poles(a, b, c_norm2: float, k: Optional[int] = None):
    """Poles theta (ascending) and residues of alpha_k from T_k (chi0_lanczos_poles, host)."""
    L = lib()
    a = _f64(a).ravel()
    b = _f64(b).ravel()
    k = a.size if k is None else int(k)
    if k > a.size or (k > 1 and b.size < k - 1):
        raise ValueError("k exceeds the coefficients given")
    bb = b if b.size else np.zeros(1)
    th = np.zeros(max(k, 1))
    r = np.zeros(max(k, 1))
    rc = L.chi0_lanczos_poles(k, _ptr(a), _ptr(bb), float(c_norm2), _ptr(th), _ptr(r))
    if rc != 0:
        raise Chi0Error(rc, "lanczos_poles")
    return th[:k], r[:k]


def debug_eigh(A):
    """Host Jacobi eigen-decomposition of the library (test hook)."""
    L = lib()
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), np.complex128)
    rc = L.chi0_debug_eigh(n, A.view(np.float64).ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                           V.view(np.float64).ctypes.data_as(_dp))
    if rc != 0:
        raise Chi0Error(rc, "debug_eigh")
    return w, V
