"""Each kernel of the chi0(w) z sequence against a host computation of its output.

Reads the library's intermediate buffers (include/chi0_debug.h) after one
chi0_apply and rebuilds the same intermediates with NumPy from the paper's
definitions (Sec. 4.2, Table t:flops):
  dV = sum_mu z_mu V_mu  ->  T = X_occ^T dV  ->  a = T X_virt, times L_EF(w)
  ->  U = a X_virt^T  ->  W = X_occ U (on the vertex pattern)  ->  n_mu = <V_mu, W>.
"""
import ctypes as C

import numpy as np
import pytest

import gpu_systems
import pins

pytestmark = pytest.mark.gpu

BUF = dict(ZIN=0, DV=1, TT=2, AT=3, UT=4, W=5, YOUT=6, BLK_NA=7, BLK_NB=8, BLK_ENT=9)


def _read(ctx, which, n, dtype=np.float64):
    L = ctx._L
    L.chi0_debug_read.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]
    out = np.zeros(n, dtype=dtype)
    rc = L.chi0_debug_read(ctx._h, BUF[which], out.ctypes.data, out.nbytes)
    assert rc == 0, ctx.last_error
    return out


def _dims(ctx):
    L = ctx._L
    d = np.zeros(10, np.int64)
    L.chi0_debug_dims.argtypes = [C.c_void_p, C.c_void_p]
    assert L.chi0_debug_dims(ctx._h, d.ctypes.data) == 0
    return d


def _blocks(sys):
    blocks = [(A, A) for A in range(sys.n_atoms)]
    off = set()
    for A, B in sys.prod_atoms:
        if B >= 0:
            off.add((int(A), int(B)))
            off.add((int(B), int(A)))
    return blocks + sorted(off)


def _close(name, got, ref, tol=1e-12):
    scale = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(got - ref)) / scale
    print(f"[stage] {name}: max rel err {err:.2e}", flush=True)
    return err < tol


# 2, 6, 18 and 40 real columns: the vertex kernels' one-, two- and four-block
# column shapes, each with a ragged last block
@pytest.mark.parametrize("name,nb", [("tiny3", 1), ("atoms12_orb9", 3), ("atoms8_orb13", 9),
                                     ("atoms12_orb9", 20)])
def test_every_stage(name, nb):
    import torch
    from paper_1005_5340_amd import chi0
    sys = gpu_systems.get(name)
    ctx = chi0.Context(0)
    ctx.set_system_from(sys)
    rng = np.random.default_rng(3)
    om = np.linspace(0.1, 1.3, nb)
    z = rng.standard_normal((nb, sys.n_prod)) + 1j * rng.standard_normal((nb, sys.n_prod))
    ctx.apply(om, sys.eps, torch.from_numpy(z).cuda())
    torch.cuda.synchronize()
    N, No, Nv, P, N_pad, No_pad, Nv_pad, P_pad, n_blk, nnzB = (int(x) for x in _dims(ctx))
    nc = 2 * nb
    mcol = No_pad * nc
    na = _read(ctx, "BLK_NA", n_blk, np.int32)
    nbk = _read(ctx, "BLK_NB", n_blk, np.int32)
    ent = _read(ctx, "BLK_ENT", n_blk, np.int64)
    blocks = _blocks(sys)
    assert len(blocks) == n_blk
    off = sys.atom_orb_offset
    Vd = pins.dense_vertices(sys)
    Xo, Xv = sys.X[:, :No], sys.X[:, No:]
    e = sys.eigenvalues
    D = e[None, No:] - e[:No, None]
    ok = True

    def to_cols(stack):   # [nb, ...] complex -> [..., nc] real
        out = np.empty(stack.shape[1:] + (nc,))
        out[..., 0::2] = np.moveaxis(stack.real, 0, -1)
        out[..., 1::2] = np.moveaxis(stack.imag, 0, -1)
        return out

    def blockrows(M):     # [nb, N, N] -> [nnzB, nc] on the pattern
        out = np.zeros((nnzB, nc))
        for k, (A, B) in enumerate(blocks):
            sub = M[:, off[A]:off[A + 1], off[B]:off[B + 1]]
            out[ent[k]:ent[k] + na[k] * nbk[k]] = to_cols(sub.reshape(nb, -1))
        return out

    def mcols(M, rows_pad):   # [nb, No, R] -> [rows_pad, No_pad*nc] with col E*nc + j
        out = np.zeros((rows_pad, No_pad, nc))
        out[:M.shape[2], :No, :] = np.transpose(to_cols(M), (1, 0, 2))
        return out.reshape(rows_pad, mcol)

    dV = np.einsum("rm,mab->rab", z, Vd)
    ok &= _close("vertex_gather", _read(ctx, "DV", nnzB * nc).reshape(nnzB, nc), blockrows(dV))
    T = np.einsum("aE,rab->rEb", Xo, dV)
    ok &= _close("occ_transform", _read(ctx, "TT", N_pad * mcol).reshape(N_pad, mcol), mcols(T, N_pad))
    zc = om[:, None, None] + 1j * sys.eps
    Lr = sys.occ_factor * (1 / (zc - D[None]) - 1 / (zc + D[None]))
    a = np.einsum("rEb,bF->rEF", T, Xv) * Lr
    ok &= _close("virt_transform_lorentz", _read(ctx, "AT", Nv_pad * mcol).reshape(Nv_pad, mcol), mcols(a, Nv_pad))
    U = np.einsum("rEF,bF->rEb", a, Xv)
    ok &= _close("virt_back", _read(ctx, "UT", N_pad * mcol).reshape(N_pad, mcol), mcols(U, N_pad))
    W = np.einsum("aE,rEb->rab", Xo, U)
    ok &= _close("occ_back", _read(ctx, "W", nnzB * nc).reshape(nnzB, nc), blockrows(W))
    n = np.einsum("mab,rab->rm", Vd, W)
    ok &= _close("vertex_contract", _read(ctx, "YOUT", P_pad * nc).reshape(P_pad, nc)[:P], to_cols(n))
    ctx.close()
    assert ok
