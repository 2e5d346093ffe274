/*
 * chi0_debug.h -- test hooks of libchi0 (not part of the stable API).
 *
 * They let a test read the library's internal device buffers after a call,
 * so that every kernel of the chi0(w) z sequence (Sec. 4.2, Table t:flops)
 * can be checked on its own against a host computation of the same
 * intermediate.  Layouts are those described in the library's internal
 * header: A batch of nb right-hand sides is nc = 2 nb real columns; row
 * strides are nc.  The buffers hold the values of the last chi0_apply or
 * solver step on the context.
 */
#ifndef CHI0_DEBUG_H
#define CHI0_DEBUG_H

#include <stdint.h>
#include "chi0.h"

#ifdef __cplusplus
extern "C" {
#endif

enum chi0_debug_buffer {
    CHI0_DBG_ZIN = 0,     /* [P_pad][nc]            operator input (after K for solver steps) */
    CHI0_DBG_DV = 1,      /* [nnzB][nc]             vertex contraction dV, block-sparse         */
    CHI0_DBG_TT = 2,      /* [N_pad][No_pad*nc]     X_occ^T dV, column m = E*nc + j            */
    CHI0_DBG_AT = 3,      /* [Nv_pad][No_pad*nc]    X_occ^T dV X_virt times the Lorentzian      */
    CHI0_DBG_UT = 4,      /* [N_pad][No_pad*nc]     back-transformed to atomic orbitals          */
    CHI0_DBG_W = 5,       /* [nnzB][nc]             X_occ U on the block pattern                 */
    CHI0_DBG_YOUT = 6,    /* [P_pad][nc]            chi0(w) z                                    */
    CHI0_DBG_BLK_NA = 7,  /* int32 [n_blk]                                                      */
    CHI0_DBG_BLK_NB = 8,  /* int32 [n_blk]                                                      */
    CHI0_DBG_BLK_ENT = 9  /* int64 [n_blk] first dV row of each block                           */
};

/* dims[0..9] = N, No, Nv, P, N_pad, No_pad, Nv_pad, P_pad, n_blk, nnzB. */
int chi0_debug_dims(const chi0_ctx *ctx, int64_t *dims);

/* Copy `bytes` bytes from the start of internal buffer `which` to host
 * memory `host` (synchronises the device).  CHI0_EINVAL if the buffer is
 * smaller or not allocated. */
int chi0_debug_read(chi0_ctx *ctx, int32_t which, void *host, int64_t bytes);

/* Warm-start network: dims[0..6] = r, n_features, width, n_outputs (2r rounded up
 * to 32), n_params, n_freq, and w_scale as a double in *w_scale.  Parameters are
 * one float vector [W1 (width x F) | b1 | W2 (width x width) | b2 | W3 (O x width) | b3],
 * weight matrices row-major with one row per output unit. */
int chi0_ws_debug_dims(const chi0_ws *ws, int64_t *dims, double *w_scale);
/* Copy the parameters to host (set = 0) or from host (set = 1). */
int chi0_ws_debug_params(chi0_ws *ws, float *host, int64_t n, int32_t set);
/* Mean squared error of the network on n (<= 256) frequencies against host
 * targets [n][n_outputs] (only the first 2r columns count) and its gradient
 * with respect to every parameter, computed by the GPU kernels (no update). */
int chi0_ws_debug_loss_grad(chi0_ws *ws, int32_t n, const double *omega, const float *target,
                            float *loss, float *grads);
/* The last chi0_lanczos with CHI0_LZ_REORTH_PARTIAL run while kernel timing
 * was on (its host reads the device decision every step): passes[j] = 1 if
 * step j ran the reorthogonalisation pass, and b_pre[j * n_drive + s] the
 * norm b_j of the three-term residual of drive s that the decision used
 * (before the pass).  Copies min(cap, steps) steps; returns the number of
 * steps recorded (0 if none).  Either pointer may be NULL. */
int chi0_debug_lz_passes(const chi0_ctx *ctx, int32_t *passes, double *b_pre, int32_t cap);

/* Host eigen-decomposition of a Hermitian n x n matrix (row-major interleaved
 * complex): eigenvalues descending in w[n], eigenvectors as columns of V. */
int chi0_debug_eigh(int32_t n, const double *A, double *w, double *V);

#ifdef __cplusplus
}
#endif
#endif
