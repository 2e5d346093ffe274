// GMRES kernels (Sec. 4.1): the Krylov basis, Gram-Schmidt orthogonalisation
// (eq. orthogonal-krylov-basis, applied twice: classical Gram-Schmidt with
// one re-orthogonalisation), the Hessenberg least-squares problem by Givens
// rotations, and the polarizability P = d . X (eq. eqpolarizability).
//
// Many (frequency, drive) points are solved at once; each occupies a slot
// with its own basis, Hessenberg matrix and solution.  A step carries one
// job per active slot (compute b = chi0 d, an Arnoldi step, or the true
// residual after a cycle).  All reductions are deterministic: fixed-order
// wavefront shuffles and a fixed tree across the four waves, no atomics.
// Inner products over C are Hermitian, <u|w> = sum conj(u) w.
#include "common.h"

namespace chi0 {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over a 256-thread workgroup; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

__device__ __forceinline__ int64_t hoff(int j) { return (int64_t)j * (j + 3) / 2; }

// Streaming load of a basis element: the basis is read once per pass and is
// far larger than the caches, so the load is marked non-temporal.
typedef double nt_dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldnt(const double2 *p) {
    const nt_dbl2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_dbl2 *>(p));
    return make_double2(v.x, v.y);
}

// ------------------------------------------------------------- gather inputs
// Operator input column pair (2q, 2q+1) <- the job's vector (zeros for b jobs).
__global__ __launch_bounds__(256)
void k_gather_jobs(const Job *__restrict__ jobs, SlotsDev sl, double *__restrict__ Vb, int nc, int P) {
    const int q = blockIdx.y, mu = blockIdx.x * 256 + threadIdx.x;
    if (mu >= sl.P_pad) return;
    const Job jb = jobs[q];
    double re = 0.0, im = 0.0;
    if (mu < P) {
        const double *src = nullptr;
        if (jb.type == JOB_ARNOLDI)
            src = sl.V + jb.slot * sl.vstride + (int64_t)jb.j * sl.P_pad * 2;
        else if (jb.type == JOB_RESID)
            src = sl.x + (int64_t)jb.slot * sl.P_pad * 2;
        if (src) {
            const double2 v = reinterpret_cast<const double2 *>(src)[mu];
            re = v.x; im = v.y;
        }
    }
    Vb[(int64_t)mu * nc + 2 * q] = re;
    Vb[(int64_t)mu * nc + 2 * q + 1] = im;
}

void launch_gather_jobs(Tracer *t, hipStream_t s, const Job *jobs, int nb, const SlotsDev &sl,
                        double *Vb, int nc, int P) {
    dim3 grid((sl.P_pad + 255) / 256, nb);
    trace_begin(t, "gather_jobs", s);
    hipLaunchKernelGGL(k_gather_jobs, grid, dim3(256), 0, s, jobs, sl, Vb, nc, P);
    trace_end(t, s);
}

// b jobs feed the drive itself to chi0 (b = chi0 d), not K times a vector.
__global__ __launch_bounds__(256)
void k_put_drive(const Job *__restrict__ jobs, const double *__restrict__ drives, int P_pad,
                 double *__restrict__ Zin, int nc, int P) {
    const int q = blockIdx.y, mu = blockIdx.x * 256 + threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_RHS || mu >= P_pad) return;
    Zin[(int64_t)mu * nc + 2 * q] = (mu < P) ? drives[(int64_t)jb.drive * P_pad + mu] : 0.0;
    Zin[(int64_t)mu * nc + 2 * q + 1] = 0.0;
}

void launch_put_drive(Tracer *t, hipStream_t s, const Job *jobs, int nb, const double *drives,
                      int P_pad, double *Zin, int nc, int P) {
    dim3 grid((P_pad + 255) / 256, nb);
    trace_begin(t, "put_drive", s);
    hipLaunchKernelGGL(k_put_drive, grid, dim3(256), 0, s, jobs, drives, P_pad, Zin, nc, P);
    trace_end(t, s);
}

// ----------------------------------------------------------------- post step
// RHS:     b = Y, x = 0 (kept if warm), r = b.   ARNOLDI: w = v_j - Y -> V[j+1].
// RESID:   r = b - (x - Y).                RHS/RESID: V[0] = r/||r||, g0 = ||r||.
// RHS/RESID also keep wa = d + K x (Zin = K x for a residual job; d alone
// after b): the solution of the transposed system A^T wa = d for the exact x,
// which the polarizability's first-order residual term uses.
__global__ __launch_bounds__(256)
void k_post_jobs(const Job *__restrict__ jobs, SlotsDev sl, const double *__restrict__ Y,
                 const double *__restrict__ Zin, const double *__restrict__ drives, int nc,
                 int P, StepStatus *__restrict__ st) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    double *V = sl.V + jb.slot * sl.vstride;
    if (jb.type == JOB_ARNOLDI) {
        const double2 *v = reinterpret_cast<const double2 *>(V + (int64_t)jb.j * vlen);
        double2 *w = reinterpret_cast<double2 *>(V + (int64_t)(jb.j + 1) * vlen);
        for (int mu = t; mu < P; mu += 256) {
            const double2 a = v[mu];
            w[mu] = make_double2(a.x - Y[(int64_t)mu * nc + 2 * q], a.y - Y[(int64_t)mu * nc + 2 * q + 1]);
        }
        return;
    }
    double2 *x = reinterpret_cast<double2 *>(sl.x + jb.slot * vlen);
    double2 *b = reinterpret_cast<double2 *>(sl.b + jb.slot * vlen);
    double2 *wa = reinterpret_cast<double2 *>(sl.w + jb.slot * vlen);
    const double *d = drives + (int64_t)jb.drive * sl.P_pad;
    double2 *v0 = reinterpret_cast<double2 *>(V);
    double ss = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double yr = Y[(int64_t)mu * nc + 2 * q], yi = Y[(int64_t)mu * nc + 2 * q + 1];
        double rr, ri;
        if (jb.type == JOB_RHS) {
            b[mu] = make_double2(yr, yi);
            if (jb.j == 0) x[mu] = make_double2(0.0, 0.0);   // else a warm start is in x
            rr = yr; ri = yi;
            wa[mu] = make_double2(d[mu], 0.0);
        } else {
            const double2 bb = b[mu], xx = x[mu];
            rr = bb.x - (xx.x - yr);
            ri = bb.y - (xx.y - yi);
            wa[mu] = make_double2(d[mu] + Zin[(int64_t)mu * nc + 2 * q], Zin[(int64_t)mu * nc + 2 * q + 1]);
        }
        v0[mu] = make_double2(rr, ri);
        ss += rr * rr + ri * ri;
    }
    const double nrm = sqrt(block_sum(ss, sh));
    const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = v0[mu];
        v0[mu] = make_double2(a.x * sc, a.y * sc);
    }
    if (t == 0) {
        double *g = sl.g + (int64_t)jb.slot * (sl.m + 1) * 2;
        g[0] = nrm; g[1] = 0.0;
        st[q].value = nrm;
        st[q].hnext = 0.0;
    }
}

void launch_post_jobs(Tracer *t, hipStream_t s, const Job *jobs, int nb, const SlotsDev &sl,
                      const double *Y, const double *Zin, const double *drives, int nc, int P,
                      StepStatus *status) {
    trace_begin(t, "post_jobs", s);
    hipLaunchKernelGGL(k_post_jobs, dim3(nb), dim3(256), 0, s, jobs, sl, Y, Zin, drives, nc, P, status);
    trace_end(t, s);
}

// ------------------------------------------------------------- Gram-Schmidt
// h_i = <v_i | w> for i <= j, w = V[j+1]; one wavefront per basis vector.
__global__ __launch_bounds__(256)
void k_cgs_dots(const Job *__restrict__ jobs, SlotsDev sl, int P) {
    const int q = blockIdx.y, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Job jb = jobs[q];
    const int i = blockIdx.x * 4 + wv;
    if (jb.type != JOB_ARNOLDI || i > jb.j) return;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double *V = sl.V + jb.slot * sl.vstride;
    const double2 *vi = reinterpret_cast<const double2 *>(V + (int64_t)i * vlen);
    const double2 *w = reinterpret_cast<const double2 *>(V + (int64_t)(jb.j + 1) * vlen);
    double re = 0.0, im = 0.0;
    for (int mu = lane; mu < P; mu += 64) {
        const double2 a = ldnt(&vi[mu]), c = w[mu];
        re += a.x * c.x + a.y * c.y;
        im += a.x * c.y - a.y * c.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        double *h = sl.hbuf + (int64_t)jb.slot * sl.hbstride;
        h[2 * i] = re;
        h[2 * i + 1] = im;
    }
}

// w -= sum_{i<=j} v_i h_i; workgroup x == 0 also adds h into column j of H.
__global__ __launch_bounds__(256)
void k_cgs_update(const Job *__restrict__ jobs, SlotsDev sl, int P, int accumulate) {
    extern __shared__ double hs[];
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int n = jb.j + 1;
    const double *h = sl.hbuf + (int64_t)jb.slot * sl.hbstride;
    for (int i = t; i < 2 * n; i += 256) hs[i] = h[i];
    __syncthreads();
    if (blockIdx.x == 0) {
        double *col = sl.H + jb.slot * sl.hstride + 2 * hoff(jb.j);
        for (int i = t; i < 2 * n; i += 256) col[i] = accumulate ? col[i] + hs[i] : hs[i];
    }
    const int mu = blockIdx.x * 256 + t;
    if (mu >= P) return;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double *V = sl.V + jb.slot * sl.vstride;
    double2 *w = reinterpret_cast<double2 *>(const_cast<double *>(V) + (int64_t)n * vlen) + mu;
    double2 acc = *w;
    for (int i = 0; i < n; ++i) {
        const double2 v = ldnt(reinterpret_cast<const double2 *>(V + (int64_t)i * vlen) + mu);
        const double hr = hs[2 * i], hi = hs[2 * i + 1];
        acc.x -= v.x * hr - v.y * hi;
        acc.y -= v.x * hi + v.y * hr;
    }
    *w = acc;
}

// ||w||, v_{j+1} = w / ||w||, then the Givens update of column j of H.
//
// Applying the earlier rotations G_i = [[c_i, s_i], [-conj(s_i), c_i]] to the
// new column h is a first-order recurrence in the running entry u:
//     r_i = c_i u_i + s_i h_{i+1},   u_{i+1} = a_i u_i + b_i,
//     a_i = -conj(s_i),  b_i = c_i h_{i+1},  u_0 = h_0,
// so the workgroup evaluates it with a parallel scan of the affine maps
// u -> a u + b (each thread composes a contiguous chunk, a Hillis-Steele
// scan combines the 256 chunk maps, then each thread replays its chunk).
struct cpx { double r, i; };
__device__ __forceinline__ cpx cmul(cpx a, cpx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cpx cadd(cpx a, cpx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cpx cdiv(cpx a, cpx b) {
    const double d = b.r * b.r + b.i * b.i;
    if (d == 0.0) return {0.0, 0.0};
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

struct GivensShared {
    cpx A[2][256], B[2][256];
    cpx ulast;
};

// Givens update of Hessenberg column j (col[0..j] from Gram-Schmidt, col[j+1]
// = hn = h_{j+1,j} >= 0): applies rotations 0..j-1, forms rotation j that
// zeroes h_{j+1,j}, updates g and returns |g_{j+1}| (valid in thread 0).
// Called by all 256 threads; tmp is scratch of >= j complex.
__device__ double givens_column(cpx *col, int j, double hn, double *cs, cpx *sn, double *g, cpx *tmp,
                                GivensShared &gs) {
    const int t = threadIdx.x;
    const int chunk = (j + 255) / 256;
    const int lo = min(j, t * chunk), hi = min(j, lo + chunk);
    cpx A = {1.0, 0.0}, B = {0.0, 0.0};          // identity map
    for (int i = lo; i < hi; ++i) {
        const cpx a = {-sn[i].r, sn[i].i};        // -conj(s_i)
        const cpx b = {cs[i] * col[i + 1].r, cs[i] * col[i + 1].i};
        B = cadd(cmul(a, B), b);                  // (a, b) o (A, B)
        A = cmul(a, A);
    }
    gs.A[0][t] = A;
    gs.B[0][t] = B;
    __syncthreads();
    int cur = 0;
    for (int o = 1; o < 256; o <<= 1) {
        cpx nA = gs.A[cur][t], nB = gs.B[cur][t];
        if (t >= o) {   // compose the earlier prefix (t-o) first, then this element
            const cpx pA = gs.A[cur][t - o], pB = gs.B[cur][t - o];
            nB = cadd(cmul(nA, pB), nB);
            nA = cmul(nA, pA);
        }
        gs.A[cur ^ 1][t] = nA;
        gs.B[cur ^ 1][t] = nB;
        cur ^= 1;
        __syncthreads();
    }
    const cpx u0 = col[0];
    cpx u = u0;
    if (t > 0) u = cadd(cmul(gs.A[cur][t - 1], u0), gs.B[cur][t - 1]);
    for (int i = lo; i < hi; ++i) {
        const cpx si = sn[i], h1 = col[i + 1];
        tmp[i] = cadd({cs[i] * u.r, cs[i] * u.i}, cmul(si, h1));
        u = cadd(cmul({-si.r, si.i}, u), {cs[i] * h1.r, cs[i] * h1.i});
    }
    if (t == 255) gs.ulast = cadd(cmul(gs.A[cur][255], u0), gs.B[cur][255]);
    __syncthreads();
    for (int i = t; i < j; i += 256) col[i] = tmp[i];
    __syncthreads();
    if (t != 0) return 0.0;
    // new rotation zeroing h_{j+1,j} = hn (real, >= 0) against u_j
    const double ar = gs.ulast.r, ai = gs.ulast.i;
    const double aa = sqrt(ar * ar + ai * ai);
    double c, sr, si, rr, ri;
    if (aa == 0.0) {
        c = 0.0; sr = 1.0; si = 0.0; rr = hn; ri = 0.0;
    } else {
        const double den = sqrt(aa * aa + hn * hn);
        c = aa / den;
        sr = (ar / aa) * hn / den;
        si = (ai / aa) * hn / den;
        rr = (ar / aa) * den;
        ri = (ai / aa) * den;
    }
    cs[j] = c;
    sn[j] = {sr, si};
    col[j] = {rr, ri};
    col[j + 1] = {0.0, 0.0};
    const double gr = g[2 * j], gi = g[2 * j + 1];
    // g_{j+1} = -conj(s) g_j, g_j = c g_j
    g[2 * (j + 1)] = -(sr * gr + si * gi);
    g[2 * (j + 1) + 1] = -(sr * gi - si * gr);
    g[2 * j] = c * gr;
    g[2 * j + 1] = c * gi;
    return sqrt(g[2 * (j + 1)] * g[2 * (j + 1)] + g[2 * (j + 1) + 1] * g[2 * (j + 1) + 1]);
}

// ||w||, v_{j+1} = w / ||w||, then the Givens update of column j of H.
//
// Applying the earlier rotations G_i = [[c_i, s_i], [-conj(s_i), c_i]] to the
// new column h is a first-order recurrence in the running entry u:
//     r_i = c_i u_i + s_i h_{i+1},   u_{i+1} = a_i u_i + b_i,
//     a_i = -conj(s_i),  b_i = c_i h_{i+1},  u_0 = h_0,
// so the workgroup evaluates it with a parallel scan of the affine maps
// u -> a u + b (each thread composes a contiguous chunk, a Hillis-Steele
// scan combines the 256 chunk maps, then each thread replays its chunk).
__global__ __launch_bounds__(256)
void k_arnoldi_finalize(const Job *__restrict__ jobs, SlotsDev sl, int P, StepStatus *__restrict__ st) {
    __shared__ double sh[4];
    __shared__ GivensShared gsh;
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int j = jb.j;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    double2 *w = reinterpret_cast<double2 *>(sl.V + jb.slot * sl.vstride + (int64_t)(j + 1) * vlen);
    double ss = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = w[mu];
        ss += a.x * a.x + a.y * a.y;
    }
    const double hn = sqrt(block_sum(ss, sh));
    const double sc = hn > 0.0 ? 1.0 / hn : 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = w[mu];
        w[mu] = make_double2(a.x * sc, a.y * sc);
    }
    cpx *col = reinterpret_cast<cpx *>(sl.H + jb.slot * sl.hstride + 2 * hoff(j));
    if (t == 0) col[j + 1] = {hn, 0.0};
    __syncthreads();
    const double est = givens_column(col, j, hn, sl.cs + (int64_t)jb.slot * sl.m,
                                     reinterpret_cast<cpx *>(sl.sn + (int64_t)jb.slot * sl.m * 2),
                                     sl.g + (int64_t)jb.slot * (sl.m + 1) * 2,
                                     reinterpret_cast<cpx *>(sl.hbuf + (int64_t)jb.slot * sl.hbstride), gsh);
    if (t == 0) {
        st[q].value = est;
        st[q].hnext = hn;
    }
}

// ------------------------------------------------ delayed reorthogonalisation
// One Arnoldi step with a single fused projection pass and a single fused
// update pass over the basis (classical Gram-Schmidt whose second pass is
// delayed by one step).  On entry V[j] holds the candidate v~_j (one pass of
// Gram-Schmidt against V_j = [v_0..v_{j-1}], unit norm) and V[j+1] holds
// z = A v~_j.  With s = V_j^H v~_j, rho^2 = |v~_j|^2 - |s|^2:
//   v_j = (v~_j - V_j s) / rho                  (finishes v_j's second pass)
//   column j-1 of H += beta~ s, h_{j,j-1} = beta~ rho   (beta~ = its provisional h_{j,j-1})
//   w' = (z - V_{j+1} V_{j+1}^H z) / rho = A v_j - V_{j+1} c,
//   c = [V_j^H z ; v_j^H z] / rho = [t / rho ; (v~_j^H z - s^H t) / rho^2]
// because A V_j s lies in span(V_{j+1}) and so drops out of the projection.
// Column j of H is set to c (exact up to the term H s / rho, of the size of
// the loss of orthogonality), and h_{j+1,j} = |w'| provisionally.  Column j-1
// is final after this step, so its Givens rotation (and the residual
// estimate for dimension j) is formed now.
//
// hbuf per slot (complex entries): s at [0, j); t at [j, 2j), overwritten by
// c_0..c_{j-1}; sigma at 2j, overwritten by c_j; tau at 2j+1, overwritten by
// rho; scratch of the Givens scan from 2j+2 (j-1 entries): 3m+4 in all.

// s_i = <v_i | v~_j>, t_i = <v_i | z> for i < j; for i = j: sigma = <v~_j|v~_j>,
// tau = <v~_j|z>.  Each wavefront takes DPW consecutive i, so v~_j and z are
// loaded once per DPW basis vectors (DPW = 4 measured fastest: 2 re-reads more
// of v~_j and z, 8 gives too few wavefronts).  With few jobs the rows are
// also split into gridDim.z ranges (at least 256 rows each) so that the step
// still fills the chip; each range writes its four sums per i to
// part[((q R + r) ld + i) 4 + c] and k_dcgs_dots_fin adds the ranges in order.
constexpr int DPW = 4;

__device__ __forceinline__ void dcgs_store_dots(double *h, int i, int j, double a0, double a1, double a2,
                                                double a3) {
    if (i < j) {
        h[2 * i] = a0; h[2 * i + 1] = a1;               // s_i
        h[2 * (j + i)] = a2; h[2 * (j + i) + 1] = a3;   // t_i
    } else {
        h[4 * j] = a0; h[4 * j + 1] = 0.0;              // sigma at 2j
        h[4 * j + 2] = a2; h[4 * j + 3] = a3;           // tau at 2j+1
    }
}

__global__ __launch_bounds__(256)
void k_dcgs_dots(const Job *__restrict__ jobs, SlotsDev sl, int P, int ld, double *__restrict__ part) {
    const int q = blockIdx.y, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = blockIdx.z, R = gridDim.z;
    const Job jb = jobs[q];
    const int i0 = (blockIdx.x * 4 + wv) * DPW;
    const int j = jb.j;
    if (jb.type != JOB_ARNOLDI || i0 > j) return;
    const int nv = min(DPW, j + 1 - i0);
    // row range of this split: multiples of 64 rows, the last range takes the rest
    const int rc = (((P + R - 1) / R) + 63) & ~63;
    const int lo = r * rc, hi = min(P, lo + rc);
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double *V = sl.V + jb.slot * sl.vstride;
    const double2 *vi = reinterpret_cast<const double2 *>(V + (int64_t)i0 * vlen);
    const double2 *vt = reinterpret_cast<const double2 *>(V + (int64_t)j * vlen);
    const double2 *z = reinterpret_cast<const double2 *>(V + (int64_t)(j + 1) * vlen);
    const int64_t vst = vlen / 2;
    double sr[DPW], si[DPW], tr[DPW], ti[DPW];
#pragma unroll
    for (int k = 0; k < DPW; ++k) sr[k] = si[k] = tr[k] = ti[k] = 0.0;
    // a group shorter than DPW repeats its last vector (its sums are not stored),
    // so the loop has no branch and its loads can be issued ahead
    int64_t off[DPW];
#pragma unroll
    for (int k = 0; k < DPW; ++k) off[k] = (int64_t)min(k, nv - 1) * vst;
    for (int mu = lo + lane; mu < hi; mu += 64) {
        const double2 b = vt[mu], c = z[mu];
#pragma unroll
        for (int k = 0; k < DPW; ++k) {
            const double2 a = ldnt(&vi[off[k] + mu]);
            sr[k] += a.x * b.x + a.y * b.y;
            si[k] += a.x * b.y - a.y * b.x;
            tr[k] += a.x * c.x + a.y * c.y;
            ti[k] += a.x * c.y - a.y * c.x;
        }
    }
#pragma unroll
    for (int k = 0; k < DPW; ++k) {
        if (k >= nv) break;
        const double a0 = wave_sum(sr[k]), a1 = wave_sum(si[k]), a2 = wave_sum(tr[k]), a3 = wave_sum(ti[k]);
        if (lane == 0) {
            const int i = i0 + k;
            if (R == 1) {
                dcgs_store_dots(sl.hbuf + (int64_t)jb.slot * sl.hbstride, i, j, a0, a1, a2, a3);
            } else {
                double *o = part + (((int64_t)q * R + r) * ld + i) * 4;
                o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3;
            }
        }
    }
}

// Adds the R row ranges of k_dcgs_dots in order and stores the sums.
__global__ __launch_bounds__(256)
void k_dcgs_dots_fin(const Job *__restrict__ jobs, SlotsDev sl, int R, int ld, const double *__restrict__ part) {
    const int q = blockIdx.y, i = blockIdx.x * 256 + threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI || i > jb.j) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int r = 0; r < R; ++r) {
        const double *o = part + (((int64_t)q * R + r) * ld + i) * 4;
        a0 += o[0]; a1 += o[1]; a2 += o[2]; a3 += o[3];
    }
    dcgs_store_dots(sl.hbuf + (int64_t)jb.slot * sl.hbstride, i, jb.j, a0, a1, a2, a3);
}

// rho, correction and Givens of column j-1, coefficients c and provisional column j.
__global__ __launch_bounds__(256)
void k_dcgs_coef(const Job *__restrict__ jobs, SlotsDev sl, StepStatus *__restrict__ st) {
    __shared__ double sh[4];
    __shared__ GivensShared gsh;
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int j = jb.j;
    cpx *h = reinterpret_cast<cpx *>(sl.hbuf + (int64_t)jb.slot * sl.hbstride);
    // |s|^2 and s^H t
    double a2 = 0.0, str = 0.0, sti = 0.0;
    for (int i = t; i < j; i += 256) {
        const cpx sv = h[i], tv = h[j + i];
        a2 += sv.r * sv.r + sv.i * sv.i;
        str += sv.r * tv.r + sv.i * tv.i;
        sti += sv.r * tv.i - sv.i * tv.r;
    }
    a2 = block_sum(a2, sh);
    str = block_sum(str, sh);
    sti = block_sum(sti, sh);
    const double sigma = h[2 * j].r;
    const cpx tau = h[2 * j + 1];
    const double r2 = sigma - a2;
    const double rho = r2 > 0.0 ? sqrt(r2) : 0.0;
    const double ir = rho > 0.0 ? 1.0 / rho : 0.0;
    double *g = sl.g + (int64_t)jb.slot * (sl.m + 1) * 2;
    double est = sqrt(g[0] * g[0] + g[1] * g[1]);
    if (j >= 1) {
        cpx *colp = reinterpret_cast<cpx *>(sl.H + jb.slot * sl.hstride + 2 * hoff(j - 1));
        const double bt = colp[j].r;                  // provisional h_{j,j-1}
        for (int i = t; i < j; i += 256) colp[i] = cadd(colp[i], {bt * h[i].r, bt * h[i].i});
        __syncthreads();
        if (t == 0) colp[j] = {bt * rho, 0.0};
        __syncthreads();
        // scratch for the scan: entries beyond 2j+1 of hbuf
        est = givens_column(colp, j - 1, bt * rho, sl.cs + (int64_t)jb.slot * sl.m,
                            reinterpret_cast<cpx *>(sl.sn + (int64_t)jb.slot * sl.m * 2), g, h + 2 * j + 2, gsh);
    }
    // c_i = t_i / rho (i < j), c_j = (tau - s^H t) / rho^2 ; stored over t, rho after it
    __syncthreads();
    cpx *colj = reinterpret_cast<cpx *>(sl.H + jb.slot * sl.hstride + 2 * hoff(j));
    for (int i = t; i < j; i += 256) {
        const cpx c = {h[j + i].r * ir, h[j + i].i * ir};
        h[j + i] = c;
        colj[i] = c;
    }
    if (t == 0) {
        const cpx cj = {(tau.r - str) * ir * ir, (tau.i - sti) * ir * ir};
        h[2 * j] = cj;
        colj[j] = cj;
        h[2 * j + 1] = {rho, 0.0};
        st[q].value = est;
    }
}

// v_j = (v~_j - V_j s) / rho and w' = z / rho - V_j c_top - v_j c_j in one pass.
// The coefficients are staged through LDS in chunks (s and c of up to 4000
// vectors do not fit at once).
constexpr int DCH = 512;

// Sums V_[i0,i1) s and V_[i0,i1) c for row mu (all threads join the LDS staging).
// The loads of UB basis vectors are issued together before their products, so
// a thread keeps UB loads in flight.
constexpr int UB = 8;
__device__ __forceinline__ void dcgs_sums(const cpx *h, int j, const double2 *vb, int64_t vst, bool act,
                                          int i0, int i1, cpx *shs, cpx *shc, double2 &as, double2 &ac) {
    const int t = threadIdx.x;
    for (int c0 = i0; c0 < i1; c0 += DCH) {
        const int n = min(DCH, i1 - c0);
        __syncthreads();
        for (int k = t; k < n; k += 256) {
            shs[k] = h[c0 + k];
            shc[k] = h[j + c0 + k];
        }
        __syncthreads();
        if (act) {
            const double2 *vp = vb + (int64_t)c0 * vst;
            int k = 0;
            for (; k + UB <= n; k += UB) {
                double2 v[UB];
#pragma unroll
                for (int u = 0; u < UB; ++u) v[u] = ldnt(&vp[(int64_t)(k + u) * vst]);
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const cpx sv = shs[k + u], cv = shc[k + u];
                    as.x += v[u].x * sv.r - v[u].y * sv.i;
                    as.y += v[u].x * sv.i + v[u].y * sv.r;
                    ac.x += v[u].x * cv.r - v[u].y * cv.i;
                    ac.y += v[u].x * cv.i + v[u].y * cv.r;
                }
            }
            for (; k < n; ++k) {
                const double2 v = ldnt(&vp[(int64_t)k * vst]);
                const cpx sv = shs[k], cv = shc[k];
                as.x += v.x * sv.r - v.y * sv.i;
                as.y += v.x * sv.i + v.y * sv.r;
                ac.x += v.x * cv.r - v.y * cv.i;
                ac.y += v.x * cv.i + v.y * cv.r;
            }
        }
    }
}

// Final formula for row mu given the sums over the whole basis V_j.
__device__ __forceinline__ void dcgs_finish(const cpx *h, int j, double *V, int64_t vlen, int mu,
                                            double2 as, double2 ac) {
    const double rho = h[2 * j + 1].r, ir = rho > 0.0 ? 1.0 / rho : 0.0;
    const cpx cj = h[2 * j];
    double2 *pv = reinterpret_cast<double2 *>(V + (int64_t)j * vlen) + mu;
    double2 *pz = reinterpret_cast<double2 *>(V + (int64_t)(j + 1) * vlen) + mu;
    const double2 vt = *pv, z = *pz;
    const double2 v = make_double2((vt.x - as.x) * ir, (vt.y - as.y) * ir);
    *pv = v;
    *pz = make_double2(z.x * ir - ac.x - (v.x * cj.r - v.y * cj.i),
                       z.y * ir - ac.y - (v.x * cj.i + v.y * cj.r));
}

__global__ __launch_bounds__(256)
void k_dcgs_update(const Job *__restrict__ jobs, SlotsDev sl, int P) {
    __shared__ cpx shs[DCH], shc[DCH];
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int mu = blockIdx.x * 256 + t;
    const bool act = mu < P;
    const int j = jb.j;
    const cpx *h = reinterpret_cast<const cpx *>(sl.hbuf + (int64_t)jb.slot * sl.hbstride);
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    double *V = sl.V + jb.slot * sl.vstride;
    const double2 *vb = reinterpret_cast<const double2 *>(V) + (act ? mu : 0);
    double2 as = make_double2(0.0, 0.0), ac = make_double2(0.0, 0.0);
    dcgs_sums(h, j, vb, vlen / 2, act, 0, j, shs, shc, as, ac);
    if (act) dcgs_finish(h, j, V, vlen, mu, as, ac);
}

// Split form for steps with few Arnoldi jobs: workgroup (x, q, g) sums basis
// vectors [g jc, (g+1) jc) of job q into part[(q G + g) P_pad + mu] (as, ac),
// then k_dcgs_update_fin adds the G partial sums in order and finishes.
__global__ __launch_bounds__(256)
void k_dcgs_update_part(const Job *__restrict__ jobs, SlotsDev sl, int P, int jc,
                        double *__restrict__ part) {
    __shared__ cpx shs[DCH], shc[DCH];
    const int q = blockIdx.y, g = blockIdx.z, G = gridDim.z, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int mu = blockIdx.x * 256 + t;
    const bool act = mu < P;
    const int j = jb.j;
    const cpx *h = reinterpret_cast<const cpx *>(sl.hbuf + (int64_t)jb.slot * sl.hbstride);
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double2 *vb = reinterpret_cast<const double2 *>(sl.V + jb.slot * sl.vstride) + (act ? mu : 0);
    double2 as = make_double2(0.0, 0.0), ac = make_double2(0.0, 0.0);
    const int i0 = min(j, g * jc), i1 = min(j, (g + 1) * jc);
    dcgs_sums(h, j, vb, vlen / 2, act, i0, i1, shs, shc, as, ac);
    if (act) {
        double2 *o = reinterpret_cast<double2 *>(part) + ((int64_t)(q * G + g) * sl.P_pad + mu) * 2;
        o[0] = as;
        o[1] = ac;
    }
}

__global__ __launch_bounds__(256)
void k_dcgs_update_fin(const Job *__restrict__ jobs, SlotsDev sl, int P, int G, const double *__restrict__ part) {
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int mu = blockIdx.x * 256 + t;
    if (mu >= P) return;
    const cpx *h = reinterpret_cast<const cpx *>(sl.hbuf + (int64_t)jb.slot * sl.hbstride);
    const double2 *o = reinterpret_cast<const double2 *>(part) + ((int64_t)q * G * sl.P_pad + mu) * 2;
    double2 as = make_double2(0.0, 0.0), ac = make_double2(0.0, 0.0);
    for (int g = 0; g < G; ++g) {
        const double2 a = o[(int64_t)g * sl.P_pad * 2], c = o[(int64_t)g * sl.P_pad * 2 + 1];
        as.x += a.x; as.y += a.y;
        ac.x += c.x; ac.y += c.y;
    }
    dcgs_finish(h, jb.j, sl.V + jb.slot * sl.vstride, (int64_t)sl.P_pad * 2, mu, as, ac);
}

// beta~ = |w'|, v~_{j+1} = w' / beta~, provisional h_{j+1,j} = beta~.
// With the error estimates on (ed.Z != NULL) also the projections of the
// vector v_j this step finished: delta_j = d . v_j and xi_j = x0^H v_j, and at
// j = 0 the start's d . x0 and |x0|^2.
__global__ __launch_bounds__(256)
void k_dcgs_norm(const Job *__restrict__ jobs, SlotsDev sl, int P, StepStatus *__restrict__ st, EpsDev ed) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    if (jb.type != JOB_ARNOLDI) return;
    const int j = jb.j;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    double2 *w = reinterpret_cast<double2 *>(sl.V + jb.slot * sl.vstride + (int64_t)(j + 1) * vlen);
    double ss = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = w[mu];
        ss += a.x * a.x + a.y * a.y;
    }
    const double hn = sqrt(block_sum(ss, sh));
    const double sc = hn > 0.0 ? 1.0 / hn : 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = w[mu];
        w[mu] = make_double2(a.x * sc, a.y * sc);
    }
    if (t == 0) {
        cpx *colj = reinterpret_cast<cpx *>(sl.H + jb.slot * sl.hstride + 2 * hoff(j));
        colj[j + 1] = {hn, 0.0};
        st[q].hnext = hn;
    }
    if (!ed.Z) return;
    const double2 *v = reinterpret_cast<const double2 *>(sl.V + jb.slot * sl.vstride + (int64_t)j * vlen);
    const double2 *x = reinterpret_cast<const double2 *>(sl.x + jb.slot * vlen);
    const double *d = ed.drives + (int64_t)jb.drive * sl.P_pad;
    double dr = 0.0, di = 0.0, xr = 0.0, xi = 0.0, pr = 0.0, pi = 0.0, xx = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = v[mu], b = x[mu];
        dr += d[mu] * a.x;
        di += d[mu] * a.y;
        xr += b.x * a.x + b.y * a.y;   // conj(x) v
        xi += b.x * a.y - b.y * a.x;
        if (j == 0) {
            pr += d[mu] * b.x;
            pi += d[mu] * b.y;
            xx += b.x * b.x + b.y * b.y;
        }
    }
    dr = block_sum(dr, sh);
    di = block_sum(di, sh);
    xr = block_sum(xr, sh);
    xi = block_sum(xi, sh);
    if (j == 0) {
        pr = block_sum(pr, sh);
        pi = block_sum(pi, sh);
        xx = block_sum(xx, sh);
    }
    if (t == 0) {
        const int64_t o = (int64_t)jb.slot * (sl.m + 1) * 2 + 2 * j;
        ed.dl[o] = dr;
        ed.dl[o + 1] = di;
        ed.xi[o] = xr;
        ed.xi[o + 1] = xi;
        if (j == 0) {
            double *S = ed.st + (int64_t)jb.slot * EPS_NS;
            S[1] = pr;
            S[2] = pi;
            S[9] = xx;
        }
    }
}

// Column c = j - 1 of Z = R^-1 from column c of R (rotated in this step):
//   z_i = -(sum_{i <= k < c} Z_ik R_kc) / R_cc  (i < c),   z_c = 1 / R_cc,
// then y_i += z_i g_c and the workgroup's partial sums of |z_i|^2,
// delta_i z_i, xi_i z_i and |y_i|^2 (rows i of this workgroup) go to
// part[(q G + x) 8 + 0..5].  Workgroup x takes rows [256 x, 256 x + 256).
constexpr int ECH = 1024;
__device__ __forceinline__ int64_t zoff(int k) { return (int64_t)k * (k + 1) / 2; }

__global__ __launch_bounds__(256)
void k_eps_column(const Job *__restrict__ jobs, SlotsDev sl, EpsDev ed, int G, double *__restrict__ part) {
    __shared__ cpx rs[ECH];
    __shared__ double sh[4];
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    const int c = jb.j - 1;
    const int i0 = blockIdx.x * 256;
    if (jb.type != JOB_ARNOLDI || c < 0 || i0 > c) return;   // uniform per workgroup
    const int i = i0 + t;
    const bool act = i <= c;
    const cpx *R = reinterpret_cast<const cpx *>(sl.H + jb.slot * sl.hstride + 2 * hoff(c));
    cpx *Z = reinterpret_cast<cpx *>(ed.Z + jb.slot * ed.zstride);
    cpx w = {0.0, 0.0};
    for (int k0 = i0; k0 < c; k0 += ECH) {    // columns below i0 meet none of these rows
        const int n = min(ECH, c - k0);
        __syncthreads();
        for (int kk = t; kk < n; kk += 256) rs[kk] = R[k0 + kk];
        __syncthreads();
        if (act)
            for (int k = max(k0, i); k < k0 + n; ++k) w = cadd(w, cmul(Z[zoff(k) + i], rs[k - k0]));
    }
    const cpx inv = cdiv({1.0, 0.0}, R[c]);
    cpx z = {0.0, 0.0}, y = {0.0, 0.0};
    double a = 0.0, br = 0.0, bi = 0.0, er = 0.0, ei = 0.0, f = 0.0;
    if (act) {
        z = i < c ? cmul({-w.r, -w.i}, inv) : inv;
        Z[zoff(c) + i] = z;
        const cpx gc = reinterpret_cast<const cpx *>(sl.g + (int64_t)jb.slot * (sl.m + 1) * 2)[c];
        cpx *yv = reinterpret_cast<cpx *>(ed.yv + (int64_t)jb.slot * sl.m * 2);
        y = cadd(i < c ? yv[i] : cpx{0.0, 0.0}, cmul(z, gc));
        yv[i] = y;
        const cpx dl = reinterpret_cast<const cpx *>(ed.dl + (int64_t)jb.slot * (sl.m + 1) * 2)[i];
        const cpx xv = reinterpret_cast<const cpx *>(ed.xi + (int64_t)jb.slot * (sl.m + 1) * 2)[i];
        const cpx b = cmul(dl, z), e = cmul(xv, z);
        a = z.r * z.r + z.i * z.i;
        br = b.r; bi = b.i; er = e.r; ei = e.i;
        f = y.r * y.r + y.i * y.i;
    }
    a = block_sum(a, sh);
    br = block_sum(br, sh);
    bi = block_sum(bi, sh);
    er = block_sum(er, sh);
    ei = block_sum(ei, sh);
    f = block_sum(f, sh);
    if (t == 0) {
        double *o = part + ((int64_t)q * G + blockIdx.x) * 8;
        o[0] = a; o[1] = br; o[2] = bi; o[3] = er; o[4] = ei; o[5] = f;
    }
}

// Adds the workgroups' partial sums in order, advances the running
// quantities and writes eps_X and eps_P of dimension j to the step's status.
__global__ __launch_bounds__(64)
void k_eps_finish(const Job *__restrict__ jobs, SlotsDev sl, EpsDev ed, int G, const double *__restrict__ part,
                  StepStatus *__restrict__ st) {
    const int q = blockIdx.x;
    const Job jb = jobs[q];
    if (threadIdx.x != 0 || jb.type != JOB_ARNOLDI) return;
    const int j = jb.j;
    double *S = ed.st + (int64_t)jb.slot * EPS_NS;
    const cpx *dl = reinterpret_cast<const cpx *>(ed.dl + (int64_t)jb.slot * (sl.m + 1) * 2);
    if (j == 0) {   // dimension 0: P and |x0|^2 came from the norm kernel
        S[0] = 0.0;
        S[3] = S[4] = 0.0;
        S[5] = 0.0;
        S[6] = dl[0].r;
        S[7] = dl[0].i;
        st[q].eps_x = st[q].eps_p = HUGE_VAL;
        return;
    }
    const int c = j - 1, n = (j + 255) / 256;
    double a = 0.0, br = 0.0, bi = 0.0, er = 0.0, ei = 0.0, f = 0.0;
    for (int k = 0; k < n; ++k) {
        const double *o = part + ((int64_t)q * G + k) * 8;
        a += o[0]; br += o[1]; bi += o[2]; er += o[3]; ei += o[4]; f += o[5];
    }
    const cpx *g = reinterpret_cast<const cpx *>(sl.g + (int64_t)jb.slot * (sl.m + 1) * 2);
    const cpx gc = g[c], gj = g[j];
    S[0] += a;
    const cpx dP = cmul(gc, {br, bi}), dS = cmul(gc, {er, ei});
    S[1] += dP.r; S[2] += dP.i;
    S[3] += dS.r; S[4] += dS.i;
    S[5] = f;
    const cpx sn = reinterpret_cast<const cpx *>(sl.sn + (int64_t)jb.slot * sl.m * 2)[c];
    const double cs = sl.cs[(int64_t)jb.slot * sl.m + c];
    const cpx phi = cadd(cmul({-sn.r, -sn.i}, {S[6], S[7]}), {cs * dl[j].r, cs * dl[j].i});
    S[6] = phi.r;
    S[7] = phi.i;
    const double zf = sqrt(S[0]);
    const double X2 = S[9] + 2.0 * S[3] + S[5];
    const double rn = sqrt(gj.r * gj.r + gj.i * gj.i);
    const cpx dr = cmul(gj, phi);
    const double pa = sqrt(S[1] * S[1] + S[2] * S[2]);
    st[q].eps_x = X2 > 0.0 ? zf * rn / sqrt(X2) : HUGE_VAL;
    st[q].eps_p = pa > 0.0 ? zf * sqrt(dr.r * dr.r + dr.i * dr.i) / pa : HUGE_VAL;
}

// Basis groups of the split update: enough workgroups to fill the chip a few
// times over, at least 32 basis vectors per group, at most 64 groups, and the
// partial sums within the scratch buffer.  A function of the step's shape only.
static int update_groups(int P, int nb, int jmax, int64_t P_pad, size_t scratch_doubles) {
    const int base = ((P + 255) / 256) * nb;
    int G = 1;
    while (G < 64 && base * G < 1024 && jmax / (2 * G) >= 32 &&
           (size_t)(2 * G) * nb * P_pad * 4 <= scratch_doubles)
        G *= 2;
    return G;
}

// Row ranges of the projection pass: split while the step has fewer than 4096
// wavefronts and each range keeps at least 256 rows; the partial sums must fit
// the scratch buffer.
static int dots_splits(int P, int nb, int jmax, size_t scratch_doubles) {
    const int64_t waves = (int64_t)((jmax + DPW) / DPW) * nb;
    int R = 1;
    while (R < 16 && waves * R < 4096 && P / (2 * R) >= 256 &&
           (size_t)(2 * R) * nb * (jmax + 1) * 4 <= scratch_doubles)
        R *= 2;
    return R;
}

void launch_dcgs(Tracer *t, hipStream_t s, const Job *jobs, int nb, int jmax, const SlotsDev &sl, int P,
                 StepStatus *status, int n_arnoldi, double sum_j1, double *scratch, size_t scratch_doubles,
                 const EpsDev *eps) {
    const int R = scratch ? dots_splits(P, nb, jmax, scratch_doubles) : 1;
    const dim3 gd((jmax + 1 + 4 * DPW - 1) / (4 * DPW), nb, R), gu((P + 255) / 256, nb);
    trace_begin(t, "dcgs_dots", s);
    hipLaunchKernelGGL(k_dcgs_dots, gd, dim3(256), 0, s, jobs, sl, P, jmax + 1, scratch);
    if (R > 1)
        hipLaunchKernelGGL(k_dcgs_dots_fin, dim3((jmax + 1 + 255) / 256, nb), dim3(256), 0, s, jobs, sl, R,
                           jmax + 1, (const double *)scratch);
    trace_end(t, s, 16.0 * P * sum_j1, 16.0 * P * (sum_j1 + 2.0 * n_arnoldi));
    trace_begin(t, "dcgs_coef", s);
    hipLaunchKernelGGL(k_dcgs_coef, dim3(nb), dim3(256), 0, s, jobs, sl, status);
    trace_end(t, s, 0.0, 16.0 * 4.0 * sum_j1);
    const int G = scratch ? update_groups(P, nb, jmax, sl.P_pad, scratch_doubles) : 1;
    trace_begin(t, "dcgs_update", s);
    if (G == 1) {
        hipLaunchKernelGGL(k_dcgs_update, gu, dim3(256), 0, s, jobs, sl, P);
    } else {
        const int jc = (jmax + G - 1) / G;
        hipLaunchKernelGGL(k_dcgs_update_part, dim3(gu.x, nb, G), dim3(256), 0, s, jobs, sl, P, jc, scratch);
        hipLaunchKernelGGL(k_dcgs_update_fin, gu, dim3(256), 0, s, jobs, sl, P, G, scratch);
    }
    trace_end(t, s, 16.0 * P * sum_j1, 16.0 * P * (sum_j1 + 3.0 * n_arnoldi));
    EpsDev none{};
    trace_begin(t, "dcgs_norm", s);
    hipLaunchKernelGGL(k_dcgs_norm, dim3(nb), dim3(256), 0, s, jobs, sl, P, status, eps ? *eps : none);
    trace_end(t, s, 4.0 * P * n_arnoldi, 16.0 * P * 2.0 * n_arnoldi);
    if (eps) {
        // partial sums in scratch: nb jobs x G workgroups x 8 (the update's
        // partial sums are consumed by now; same stream)
        const int G = (jmax + 255) / 256 > 0 ? (jmax + 255) / 256 : 1;
        trace_begin(t, "eps_estimates", s);
        hipLaunchKernelGGL(k_eps_column, dim3(G, nb), dim3(256), 0, s, jobs, sl, *eps, G, scratch);
        hipLaunchKernelGGL(k_eps_finish, dim3(nb), dim3(64), 0, s, jobs, sl, *eps, G,
                           (const double *)scratch, status);
        trace_end(t, s, 0.0, 8.0 * (double)jmax * jmax * n_arnoldi);
    }
}

void launch_arnoldi(Tracer *t, hipStream_t s, const Job *jobs, int nb, int jmax,
                    const SlotsDev &sl, int P, StepStatus *status, int n_arnoldi, double sum_j1) {
    const dim3 gd((jmax + 1 + 3) / 4, nb), gu((P + 255) / 256, nb);
    const size_t shm = (size_t)(jmax + 1) * 2 * sizeof(double);
    for (int pass = 0; pass < 2; ++pass) {
        trace_begin(t, "cgs_dots", s);
        hipLaunchKernelGGL(k_cgs_dots, gd, dim3(256), 0, s, jobs, sl, P);
        trace_end(t, s, 8.0 * P * sum_j1, 16.0 * P * (sum_j1 + n_arnoldi));
        trace_begin(t, "cgs_update", s);
        hipLaunchKernelGGL(k_cgs_update, gu, dim3(256), shm, s, jobs, sl, P, pass);
        trace_end(t, s, 8.0 * P * sum_j1, 16.0 * P * (sum_j1 + 2.0 * n_arnoldi));
    }
    trace_begin(t, "arnoldi_finalize", s);
    hipLaunchKernelGGL(k_arnoldi_finalize, dim3(nb), dim3(256), 0, s, jobs, sl, P, status);
    trace_end(t, s, 4.0 * P * n_arnoldi, 16.0 * P * 2.0 * n_arnoldi);
}

// ------------------------------------------------------- end of a GMRES cycle
// y = R^{-1} g over the cycle length L = jobs[q].j (R = rotated Hessenberg,
// column i of R is column i of the packed H).  Blocked back substitution:
// the 32 x 32 diagonal block is solved by wavefront 0 from registers (rows in
// lanes, the pivot broadcast by shuffles), then all threads subtract the
// block's contribution from the rows above it.
__device__ __forceinline__ cpx cshfl(cpx v, int src) { return {__shfl(v.r, src), __shfl(v.i, src)}; }

constexpr int TSB = 32;    // rows of a diagonal block solved by one wavefront
constexpr int TPW = 256;   // rows of a panel (one launch pair per panel)

// y[0, L) = g[0, L): the working right-hand side of the back substitution.
__global__ __launch_bounds__(256)
void k_tri_init(const Job *__restrict__ jobs, SlotsDev sl) {
    const int q = blockIdx.y, i = blockIdx.x * 256 + threadIdx.x;
    const Job jb = jobs[q];
    if (i >= jb.j) return;
    const cpx *g = reinterpret_cast<const cpx *>(sl.g + (int64_t)jb.slot * (sl.m + 1) * 2);
    reinterpret_cast<cpx *>(sl.y + (int64_t)jb.slot * sl.m * 2)[i] = g[i];
}

// Panel p (from the bottom) of y = R^{-1} y: rows [lo, hi), hi = L - p TPW.
// The rows below hi are solved and already subtracted from these rows, so
// the panel is a triangular solve with its own diagonal block: 32 x 32
// blocks from the bottom, each solved by wavefront 0 from registers (rows in
// lanes, the pivot broadcast by shuffles), then subtracted by all threads
// from the panel's rows above it.
__global__ __launch_bounds__(256)
void k_tri_diag(const Job *__restrict__ jobs, SlotsDev sl, int p) {
    __shared__ cpx ys[TPW];
    __shared__ cpx yb[TSB];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    const int hi = jb.j - p * TPW;
    if (hi <= 0) return;
    const int lo = hi > TPW ? hi - TPW : 0;
    const double *H = sl.H + jb.slot * sl.hstride;
    cpx *y = reinterpret_cast<cpx *>(sl.y + (int64_t)jb.slot * sl.m * 2);
    for (int i = lo + t; i < hi; i += 256) ys[i - lo] = y[i];
    __syncthreads();
    for (int bh = hi; bh > lo; bh -= TSB) {
        const int bl = bh - TSB > lo ? bh - TSB : lo;   // block rows [bl, bh)
        const int b0 = bh - TSB;                        // lane t holds row b0 + t
        if (t < 64) {
            const int r = b0 + t;
            const bool rv = t < TSB && r >= bl;
            cpx v = rv ? ys[r - lo] : cpx{0.0, 0.0};
            cpx R[TSB];
#pragma unroll
            for (int s2 = 0; s2 < TSB; ++s2) {
                const int i = b0 + s2;
                const cpx *coli = reinterpret_cast<const cpx *>(H + 2 * hoff(i < bl ? bl : i));
                R[s2] = (rv && i >= bl && r <= i) ? coli[r] : cpx{0.0, 0.0};
            }
            // each lane inverts its own diagonal entry, so the sequential
            // sweep below multiplies instead of dividing
            cpx dinv = {0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < TSB; ++s2)
                if (t == s2) dinv = cdiv({1.0, 0.0}, R[s2]);
#pragma unroll
            for (int s2 = TSB - 1; s2 >= 0; --s2) {
                if (b0 + s2 < bl) continue;                // uniform
                const cpx yi = cmul(cshfl(v, s2), cshfl(dinv, s2));
                if (t < s2) {
                    const cpx pr = cmul(R[s2], yi);
                    v = {v.r - pr.r, v.i - pr.i};
                }
                if (t == 0) yb[s2] = yi;
            }
            // rows of the block's top part outside the panel contribute nothing
            if (t < TSB && b0 + t < bl) yb[t] = {0.0, 0.0};
        }
        __syncthreads();
        for (int s2 = t; s2 < TSB; s2 += 256)
            if (b0 + s2 >= bl) ys[b0 + s2 - lo] = yb[s2];
        for (int k = lo + t; k < bl; k += 256) {
            cpx acc = ys[k - lo];
            cpx rk[TSB];
#pragma unroll
            for (int s2 = 0; s2 < TSB; ++s2) {   // loads first (columns below bl have yb = 0)
                const int i = b0 + s2 < bl ? bl : b0 + s2;
                rk[s2] = reinterpret_cast<const cpx *>(H + 2 * hoff(i))[k];
            }
#pragma unroll
            for (int s2 = 0; s2 < TSB; ++s2) {
                const cpx pr = cmul(rk[s2], yb[s2]);
                acc = {acc.r - pr.r, acc.i - pr.i};
            }
            ys[k - lo] = acc;
        }
        __syncthreads();
    }
    for (int i = lo + t; i < hi; i += 256) y[i] = ys[i - lo];
}

// Rows above panel p: y[k] -= sum_{i in [lo, hi)} R[k][i] y[i] for k < lo,
// spread over many workgroups (the panel's R columns are read once).  A
// workgroup takes 64 rows; its wavefront w sums the panel's columns
// [lo + 64 w, lo + 64 w + 64), eight loads in flight per lane, and wavefront 0
// adds the four partial sums in order.
__global__ __launch_bounds__(256)
void k_tri_update(const Job *__restrict__ jobs, SlotsDev sl, int p) {
    __shared__ cpx ys[TPW];
    __shared__ cpx part[4][64];
    const int q = blockIdx.y, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const Job jb = jobs[q];
    const int hi = jb.j - p * TPW;
    const int lo = hi > TPW ? hi - TPW : 0;
    if (lo <= 0 || blockIdx.x * 64 >= lo) return;   // uniform per workgroup
    const double *H = sl.H + jb.slot * sl.hstride;
    cpx *y = reinterpret_cast<cpx *>(sl.y + (int64_t)jb.slot * sl.m * 2);
    for (int i = lo + t; i < hi; i += 256) ys[i - lo] = y[i];
    __syncthreads();
    const int k = blockIdx.x * 64 + lane;
    const int kk = k < lo ? k : lo - 1;             // rows past lo read a valid row, unused
    cpx acc = {0.0, 0.0};
    const int c0 = wv * (TPW / 4);                  // hi - lo == TPW here (lo > 0)
    for (int c = c0; c < c0 + TPW / 4; c += 8) {
        cpx rk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) rk[u] = reinterpret_cast<const cpx *>(H + 2 * hoff(lo + c + u))[kk];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const cpx pr = cmul(rk[u], ys[c + u]);
            acc = {acc.r + pr.r, acc.i + pr.i};
        }
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && k < lo) {
        cpx sum = y[k];
#pragma unroll
        for (int w = 0; w < 4; ++w) sum = {sum.r - part[w][lane].r, sum.i - part[w][lane].i};
        y[k] = sum;
    }
}

// x += sum_{i<L} v_i y_i, the coefficients staged through LDS in chunks.
constexpr int XCH = 1024;
__global__ __launch_bounds__(256)
void k_xupdate(const Job *__restrict__ jobs, SlotsDev sl, int P) {
    __shared__ cpx ys[XCH];
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    const int L = jb.j;
    const cpx *y = reinterpret_cast<const cpx *>(sl.y + (int64_t)jb.slot * sl.m * 2);
    const int mu = blockIdx.x * 256 + t;
    const bool act = mu < P;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double *V = sl.V + jb.slot * sl.vstride;
    double2 *x = reinterpret_cast<double2 *>(sl.x + jb.slot * vlen) + (act ? mu : 0);
    double2 acc = act ? *x : make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < L; c0 += XCH) {
        const int n = min(XCH, L - c0);
        __syncthreads();
        for (int k = t; k < n; k += 256) ys[k] = y[c0 + k];
        __syncthreads();
        if (act)
            for (int k = 0; k < n; ++k) {
                const double2 v = ldnt(reinterpret_cast<const double2 *>(V + (int64_t)(c0 + k) * vlen) + mu);
                acc.x += v.x * ys[k].r - v.y * ys[k].i;
                acc.y += v.x * ys[k].i + v.y * ys[k].r;
            }
    }
    if (act) *x = acc;
}

void launch_update_x(Tracer *t, hipStream_t s, const Job *jobs, int n, int jmax,
                     const SlotsDev &sl, int P, double sum_L) {
    trace_begin(t, "trisolve", s);
    hipLaunchKernelGGL(k_tri_init, dim3((jmax + 255) / 256, n), dim3(256), 0, s, jobs, sl);
    for (int p = 0; p * TPW < jmax; ++p) {
        hipLaunchKernelGGL(k_tri_diag, dim3(n), dim3(256), 0, s, jobs, sl, p);
        const int above = jmax - (p + 1) * TPW;
        if (above > 0)
            hipLaunchKernelGGL(k_tri_update, dim3((above + 63) / 64, n), dim3(256), 0, s, jobs, sl, p);
    }
    trace_end(t, s);
    trace_begin(t, "x_update", s);
    hipLaunchKernelGGL(k_xupdate, dim3((P + 255) / 256, n), dim3(256), 0, s, jobs, sl, P);
    trace_end(t, s, 8.0 * P * sum_L, 16.0 * P * (sum_L + 2.0 * n));
}

// ------------------------------------------------------------ polarizability
// alpha[point][k] = -d_k . x  (bilinear, eq. eqpolarizability with alpha = -P);
// jobs[q].j holds the point index, whose drive is i = point % n_drive.
//
// Residual term (Sec. 4.1 writes the error of P as d . A^-1 r): A^-T d_k is
// d_k + K x_k exactly at the solution x_k of drive k, because chi0 and K are
// complex symmetric (A^T = 1 - K chi0 and (1 - K chi0)(d + K x) = d when
// (1 - chi0 K) x = chi0 d).  So P_ki = d_k . x_i + (d_k + K x_k) . r_i holds
// up to (K (x_k* - x_k)) . r_i, second order in the residuals.  With
// `correct` the diagonal term (k = i, both factors from this slot: r =
// g_0 V_0 and wa = d_i + K x_i of its last FP64 true residual) is added here;
// Rst / Wst keep r and wa of the point for the cross terms (k != i).
__global__ __launch_bounds__(256)
void k_alpha(const Job *__restrict__ jobs, SlotsDev sl, const double *__restrict__ drives,
             int n_drive, int P_pad, int P, int correct, double *__restrict__ Rst,
             double *__restrict__ Wst, double *__restrict__ out) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    const int64_t p = jb.j;
    const double2 *x = reinterpret_cast<const double2 *>(sl.x + (int64_t)jb.slot * P_pad * 2);
    for (int k = 0; k < n_drive; ++k) {
        const double *d = drives + (int64_t)k * P_pad;
        double re = 0.0, im = 0.0;
        for (int mu = t; mu < P; mu += 256) {
            const double2 a = x[mu];
            re += d[mu] * a.x;
            im += d[mu] * a.y;
        }
        re = block_sum(re, sh);
        im = block_sum(im, sh);
        if (t == 0) {
            out[(p * n_drive + k) * 2] = -re;
            out[(p * n_drive + k) * 2 + 1] = -im;
        }
    }
    if (!correct) return;
    const double2 *v0 = reinterpret_cast<const double2 *>(sl.V + jb.slot * sl.vstride);
    const double2 *wa = reinterpret_cast<const double2 *>(sl.w + (int64_t)jb.slot * P_pad * 2);
    const double g0 = sl.g[(int64_t)jb.slot * (sl.m + 1) * 2];   // ||r||; v0 = r / ||r||
    double re = 0.0, im = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 v = v0[mu], w = wa[mu];
        const double2 r = make_double2(g0 * v.x, g0 * v.y);
        re += w.x * r.x - w.y * r.y;
        im += w.x * r.y + w.y * r.x;
        if (Rst) {
            reinterpret_cast<double2 *>(Rst)[p * P + mu] = r;
            reinterpret_cast<double2 *>(Wst)[p * P + mu] = w;
        }
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (t == 0) {
        const int64_t i = p % n_drive;
        out[(p * n_drive + i) * 2] -= re;
        out[(p * n_drive + i) * 2 + 1] -= im;
    }
}

void launch_alpha(Tracer *t, hipStream_t s, const Job *jobs, int n, const SlotsDev &sl,
                  const double *drives, int n_drive, int P_pad, int P, bool correct,
                  double *Rst, double *Wst, double *alpha_out) {
    trace_begin(t, "alpha", s);
    hipLaunchKernelGGL(k_alpha, dim3(n), dim3(256), 0, s, jobs, sl, drives, n_drive, P_pad, P, correct ? 1 : 0,
                       Rst, Wst, alpha_out);
    trace_end(t, s);
}

// Cross-drive residual terms: one workgroup per (frequency w, drive k, drive i != k).
__global__ __launch_bounds__(256)
void k_alpha_cross(int n_drive, int P, const double *__restrict__ Rst, const double *__restrict__ Wst,
                   double *__restrict__ out) {
    __shared__ double sh[4];
    const int w = blockIdx.x, k = blockIdx.y, i = blockIdx.z, t = threadIdx.x;
    if (k == i) return;
    const int64_t pi = (int64_t)w * n_drive + i, pk = (int64_t)w * n_drive + k;
    const double2 *r = reinterpret_cast<const double2 *>(Rst) + pi * P;
    const double2 *wa = reinterpret_cast<const double2 *>(Wst) + pk * P;
    double re = 0.0, im = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = wa[mu], b = r[mu];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (t == 0) {
        out[(pi * n_drive + k) * 2] -= re;
        out[(pi * n_drive + k) * 2 + 1] -= im;
    }
}

void launch_alpha_cross(Tracer *t, hipStream_t s, int n_omega, int n_drive, int P, const double *Rst,
                        const double *Wst, double *alpha_out) {
    if (n_drive < 2 || n_omega < 1) return;
    trace_begin(t, "alpha_cross", s);
    hipLaunchKernelGGL(k_alpha_cross, dim3(n_omega, n_drive, n_drive), dim3(256), 0, s, n_drive, P, Rst, Wst,
                       alpha_out);
    trace_end(t, s);
}

// ------------------------------------------------------------ apply helpers
__global__ __launch_bounds__(256)
void k_rows_to_cols(const double *__restrict__ z, int P, double *__restrict__ Zin, int nc) {
    const int r = blockIdx.y, mu = blockIdx.x * 256 + threadIdx.x;
    if (mu >= P) return;
    const double2 v = reinterpret_cast<const double2 *>(z + (int64_t)r * P * 2)[mu];
    Zin[(int64_t)mu * nc + 2 * r] = v.x;
    Zin[(int64_t)mu * nc + 2 * r + 1] = v.y;
}

__global__ __launch_bounds__(256)
void k_cols_to_rows(const double *__restrict__ Y, int P, int nc, double *__restrict__ out) {
    const int r = blockIdx.y, mu = blockIdx.x * 256 + threadIdx.x;
    if (mu >= P) return;
    reinterpret_cast<double2 *>(out + (int64_t)r * P * 2)[mu] =
        make_double2(Y[(int64_t)mu * nc + 2 * r], Y[(int64_t)mu * nc + 2 * r + 1]);
}

void launch_rows_to_cols(Tracer *t, hipStream_t s, const double *z, int nb, int P,
                         double *Zin, int nc) {
    trace_begin(t, "rows_to_cols", s);
    hipLaunchKernelGGL(k_rows_to_cols, dim3((P + 255) / 256, nb), dim3(256), 0, s, z, P, Zin, nc);
    trace_end(t, s);
}

void launch_cols_to_rows(Tracer *t, hipStream_t s, const double *Y, int nb, int P, int nc,
                         double *out) {
    trace_begin(t, "cols_to_rows", s);
    hipLaunchKernelGGL(k_cols_to_rows, dim3((P + 255) / 256, nb), dim3(256), 0, s, Y, P, nc, out);
    trace_end(t, s);
}

__global__ __launch_bounds__(256) void k_zero(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0.0;
}

void launch_zero(Tracer *t, hipStream_t s, double *p, int64_t n) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    trace_begin(t, "zero", s);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    trace_end(t, s);
}

}  // namespace chi0
