// Two-sided (biorthogonal) Lanczos recursion on A = 1 - chi0(w) K for the
// polarizability P = d^T A^-1 chi0 d (the Krylov method that the Sec. 4
// introduction says the authors used before the solve of eq. sle).  Right
// start b = chi0 d, left start d, bilinear form x^T y (no conjugate):
//
//   beta_1 = sqrt(d^T b), v_1 = b / beta_1, w_1 = d / beta_1,
//   alpha_k = w_k^T A v_k,
//   r = A v_k - alpha_k v_k - beta_k v_{k-1},  s = A^T w_k - alpha_k w_k - beta_k w_{k-1},
//   beta_{k+1} = sqrt(s^T r),  v_{k+1} = r / beta_{k+1},  w_{k+1} = s / beta_{k+1},
//
// with A v = v - chi0 (K v) and A^T w = w - K (chi0 w) (chi0 and K symmetric).
// The operator products run in the chi0 and K kernels; the kernels here do
// the per-point vector work, one 256-thread workgroup per point, with
// fixed-order reductions.  Vectors are operator columns: complex column q of
// an array with leading dimension ld (real columns 2q, 2q+1), rows mu < P
// (rows P..P_pad stay zero).
#include "common.h"

namespace chi0 {

namespace {

__device__ __forceinline__ double bl_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the 256-thread workgroup in a fixed order; every thread gets it.
__device__ __forceinline__ double bl_block_sum(double v, double *sh) {
    v = bl_wave_sum(v);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

struct cplx {
    double r, i;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    const double den = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / den, (a.i * b.r - a.r * b.i) / den};
}
// principal square root
__device__ __forceinline__ cplx csqrt_p(cplx a) {
    const double m = sqrt(a.r * a.r + a.i * a.i);
    if (m == 0.0) return {0.0, 0.0};
    const double re = sqrt(0.5 * (m + a.r));
    const double im = sqrt(0.5 * (m - a.r));
    return {re, a.i < 0.0 ? -im : im};
}
__device__ __forceinline__ cplx cld(const double *p, int64_t mu, int ld_, int q) {
    return {p[mu * ld_ + 2 * q], p[mu * ld_ + 2 * q + 1]};
}
__device__ __forceinline__ void cst(double *p, int64_t mu, int ld_, int q, cplx v) {
    p[mu * ld_ + 2 * q] = v.r;
    p[mu * ld_ + 2 * q + 1] = v.i;
}

}  // namespace

// Start of each point q: from b = chi0 d (Yb, complex column q, leading
// dimension ldb) and its drive d (real row D[drive(q)]), beta_1 = sqrt(d^T b),
// v_1 = b / beta_1, w_1 = d / beta_1, v_0 = w_0 = 0; |b| into bnorm[q].  A zero
// b (a zero drive) or d^T b = 0 marks the point finished before its first
// step (flag -1) and leaves its vectors zero.
__global__ __launch_bounds__(256)
void k_bl_init(int P, int npts, int p0, int n_drive, const double *__restrict__ D, int P_pad,
               const double *__restrict__ Yb, int ldb, double *__restrict__ V1, double *__restrict__ W1,
               double *__restrict__ V0, double *__restrict__ W0, int ld, double *__restrict__ beta,
               int ldbeta, double *__restrict__ bnorm, int *__restrict__ flag) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const double *d = D + (int64_t)((p0 + q) % n_drive) * P_pad;
    double sr = 0.0, si = 0.0, nb = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const cplx b = cld(Yb, mu, ldb, q);
        sr += d[mu] * b.r;
        si += d[mu] * b.i;
        nb += b.r * b.r + b.i * b.i;
    }
    sr = bl_block_sum(sr, sh);
    si = bl_block_sum(si, sh);
    nb = bl_block_sum(nb, sh);
    const cplx b1 = csqrt_p({sr, si});
    const bool ok = nb > 0.0 && (b1.r != 0.0 || b1.i != 0.0) && isfinite(b1.r) && isfinite(b1.i);
    if (t == 0) {
        beta[(int64_t)q * ldbeta] = b1.r;
        beta[(int64_t)q * ldbeta + 1] = b1.i;
        bnorm[q] = sqrt(nb);
        flag[q] = ok ? 0 : -1;
    }
    for (int mu = t; mu < P; mu += 256) {
        const cplx b = cld(Yb, mu, ldb, q);
        cst(V1, mu, ld, q, ok ? cdiv(b, b1) : cplx{0.0, 0.0});
        cst(W1, mu, ld, q, ok ? cdiv({d[mu], 0.0}, b1) : cplx{0.0, 0.0});
        cst(V0, mu, ld, q, {0.0, 0.0});
        cst(W0, mu, ld, q, {0.0, 0.0});
    }
}

// Operator input of the start: complex column q of Zin (leading dimension 2 np)
// <- the drive of point p0 + q (real), rows >= P zero.
__global__ __launch_bounds__(256)
void k_bl_drives(int P, int P_pad, int np, int p0, int n_drive, const double *__restrict__ D,
                 double *__restrict__ Zin) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)P_pad * 2 * np) return;
    const int64_t mu = idx / (2 * np);
    const int c = (int)(idx % (2 * np)), q = c >> 1;
    Zin[idx] = ((c & 1) || mu >= P) ? 0.0 : D[(int64_t)((p0 + q) % n_drive) * P_pad + mu];
}

// Operator input of a step: Zin columns [0, nc) <- K v (KV), [nc, 2 nc) <- w (W1);
// rows < P_pad (Zin has leading dimension 2 nc).
__global__ __launch_bounds__(256)
void k_bl_pack(int P_pad, int nc, const double *__restrict__ KV, const double *__restrict__ W1,
               double *__restrict__ Zin) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)P_pad * 2 * nc) return;
    const int64_t mu = idx / (2 * nc);
    const int c = (int)(idx % (2 * nc));
    Zin[idx] = c < nc ? KV[mu * nc + c] : W1[mu * nc + c - nc];
}

// CW <- chi0 w: columns [nc, 2 nc) of Yout (leading dimension 2 nc), rows >= P zero.
__global__ __launch_bounds__(256)
void k_bl_unpack(int P, int P_pad, int nc, const double *__restrict__ Yout, double *__restrict__ CW) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)P_pad * nc) return;
    const int64_t mu = idx / nc;
    const int c = (int)(idx % nc);
    CW[idx] = mu < P ? Yout[mu * 2 * nc + nc + c] : 0.0;
}

// Step k of each unfinished point q (flag[q] == 0):
//   A v = v - Y (Y = chi0 K v: column q of Yout, leading dimension 2 ld),
//   A^T w = w - KCW,
//   alpha_k = w^T A v;  r = A v - alpha_k v - beta_k V0;  s = A^T w - alpha_k w - beta_k W0;
//   beta_{k+1} = sqrt(s^T r);  V0 <- r / beta_{k+1},  W0 <- s / beta_{k+1}.
// The caller then swaps (V0, V1) and (W0, W1).  Records alpha_k (alpha[q][k]),
// beta_{k+1} (beta[q][k + 1]) and |r| (rnorm[q][k]).  If s^T r == 0, beta_{k+1}
// is not finite, or r or s vanishes to rounding (|r| <= 1e-13 |A v|: an
// invariant subspace), flag[q] = 2 + k (breakdown after step k) and the
// vectors are left unscaled.
__global__ __launch_bounds__(256)
void k_bl_step(int P, int k, const double *__restrict__ Yout, const double *__restrict__ KCW,
               const double *__restrict__ V1, const double *__restrict__ W1, double *__restrict__ V0,
               double *__restrict__ W0, int ld, double *__restrict__ alpha, int ldalpha,
               double *__restrict__ beta, int ldbeta, double *__restrict__ rnorm, int ldrn,
               int *__restrict__ flag) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    if (flag[q] != 0) return;
    const int ldy = 2 * ld;
    // alpha_k = w^T (v - Y)
    double ar = 0.0, ai = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const cplx v = cld(V1, mu, ld, q), y = cld(Yout, mu, ldy, q), w = cld(W1, mu, ld, q);
        const cplx av = {v.r - y.r, v.i - y.i};
        const cplx p = cmul(w, av);
        ar += p.r;
        ai += p.i;
    }
    ar = bl_block_sum(ar, sh);
    ai = bl_block_sum(ai, sh);
    const cplx a = {ar, ai};
    const cplx bk = {beta[(int64_t)q * ldbeta + 2 * k], beta[(int64_t)q * ldbeta + 2 * k + 1]};
    const cplx bkk = k > 0 ? bk : cplx{0.0, 0.0};
    double dr = 0.0, di = 0.0, rr = 0.0, ss = 0.0, avn = 0.0, awn = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const cplx v = cld(V1, mu, ld, q), y = cld(Yout, mu, ldy, q), w = cld(W1, mu, ld, q);
        const cplx kc = cld(KCW, mu, ld, q);
        const cplx av = {v.r - y.r, v.i - y.i};
        const cplx aw = {w.r - kc.r, w.i - kc.i};
        const cplx av_ = cmul(a, v), aw_ = cmul(a, w);
        const cplx bv = cmul(bkk, cld(V0, mu, ld, q)), bw = cmul(bkk, cld(W0, mu, ld, q));
        const cplx r = {av.r - av_.r - bv.r, av.i - av_.i - bv.i};
        const cplx s = {aw.r - aw_.r - bw.r, aw.i - aw_.i - bw.i};
        cst(V0, mu, ld, q, r);
        cst(W0, mu, ld, q, s);
        const cplx sr = cmul(s, r);
        dr += sr.r;
        di += sr.i;
        rr += r.r * r.r + r.i * r.i;
        ss += s.r * s.r + s.i * s.i;
        avn += av.r * av.r + av.i * av.i;
        awn += aw.r * aw.r + aw.i * aw.i;
    }
    dr = bl_block_sum(dr, sh);
    di = bl_block_sum(di, sh);
    rr = bl_block_sum(rr, sh);
    ss = bl_block_sum(ss, sh);
    avn = bl_block_sum(avn, sh);
    awn = bl_block_sum(awn, sh);
    const cplx bn = csqrt_p({dr, di});
    const bool invariant = sqrt(rr) <= 1e-13 * sqrt(avn) || sqrt(ss) <= 1e-13 * sqrt(awn);
    const bool brk = (dr == 0.0 && di == 0.0) || !isfinite(bn.r) || !isfinite(bn.i) || invariant;
    if (t == 0) {
        alpha[(int64_t)q * ldalpha + 2 * k] = a.r;
        alpha[(int64_t)q * ldalpha + 2 * k + 1] = a.i;
        beta[(int64_t)q * ldbeta + 2 * (k + 1)] = brk ? 0.0 : bn.r;
        beta[(int64_t)q * ldbeta + 2 * (k + 1) + 1] = brk ? 0.0 : bn.i;
        rnorm[(int64_t)q * ldrn + k] = sqrt(rr);
        if (brk) flag[q] = 2 + k;
    }
    if (brk) return;
    // every thread rescales the entries it wrote itself above
    for (int mu = t; mu < P; mu += 256) {
        cst(V0, mu, ld, q, cdiv(cld(V0, mu, ld, q), bn));
        cst(W0, mu, ld, q, cdiv(cld(W0, mu, ld, q), bn));
    }
}

void launch_bl_init(hipStream_t s, int P, int npts, int p0, int n_drive, const double *D, int P_pad,
                    const double *Yb, int ldb, double *V1, double *W1, double *V0, double *W0, int ld,
                    double *beta, int ldbeta, double *bnorm, int *flag) {
    hipLaunchKernelGGL(k_bl_init, dim3(npts), dim3(256), 0, s, P, npts, p0, n_drive, D, P_pad, Yb, ldb, V1, W1,
                       V0, W0, ld, beta, ldbeta, bnorm, flag);
}

void launch_bl_drives(hipStream_t s, int P, int P_pad, int np, int p0, int n_drive, const double *D, double *Zin) {
    const int64_t n = (int64_t)P_pad * 2 * np;
    hipLaunchKernelGGL(k_bl_drives, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, P_pad, np, p0, n_drive,
                       D, Zin);
}

void launch_bl_pack(hipStream_t s, int P_pad, int nc, const double *KV, const double *W1, double *Zin) {
    const int64_t n = (int64_t)P_pad * 2 * nc;
    hipLaunchKernelGGL(k_bl_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P_pad, nc, KV, W1, Zin);
}

void launch_bl_unpack(hipStream_t s, int P, int P_pad, int nc, const double *Yout, double *CW) {
    const int64_t n = (int64_t)P_pad * nc;
    hipLaunchKernelGGL(k_bl_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, P_pad, nc, Yout, CW);
}

void launch_bl_step(hipStream_t s, int npts, int P, int k, const double *Yout, const double *KCW,
                    const double *V1, const double *W1, double *V0, double *W0, int ld, double *alpha,
                    int ldalpha, double *beta, int ldbeta, double *rnorm, int ldrn, int *flag) {
    hipLaunchKernelGGL(k_bl_step, dim3(npts), dim3(256), 0, s, P, k, Yout, KCW, V1, W1, V0, W0, ld, alpha,
                       ldalpha, beta, ldbeta, rnorm, ldrn, flag);
}

}  // namespace chi0
