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
// RHS:     b = Y, x = 0, r = b.            ARNOLDI: w = v_j - Y -> V[j+1].
// RESID:   r = b - (x - Y).                RHS/RESID: V[0] = r/||r||, g0 = ||r||.
__global__ __launch_bounds__(256)
void k_post_jobs(const Job *__restrict__ jobs, SlotsDev sl, const double *__restrict__ Y, int nc,
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
    double2 *v0 = reinterpret_cast<double2 *>(V);
    double ss = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double yr = Y[(int64_t)mu * nc + 2 * q], yi = Y[(int64_t)mu * nc + 2 * q + 1];
        double rr, ri;
        if (jb.type == JOB_RHS) {
            b[mu] = make_double2(yr, yi);
            x[mu] = make_double2(0.0, 0.0);
            rr = yr; ri = yi;
        } else {
            const double2 bb = b[mu], xx = x[mu];
            rr = bb.x - (xx.x - yr);
            ri = bb.y - (xx.y - yi);
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
                      const double *Y, int nc, int P, StepStatus *status) {
    trace_begin(t, "post_jobs", s);
    hipLaunchKernelGGL(k_post_jobs, dim3(nb), dim3(256), 0, s, jobs, sl, Y, nc, P, status);
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
        const double2 a = vi[mu], c = w[mu];
        re += a.x * c.x + a.y * c.y;
        im += a.x * c.y - a.y * c.x;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        double *h = sl.hbuf + (int64_t)jb.slot * (sl.m + 1) * 2;
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
    const double *h = sl.hbuf + (int64_t)jb.slot * (sl.m + 1) * 2;
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
        const double2 v = reinterpret_cast<const double2 *>(V + (int64_t)i * vlen)[mu];
        const double hr = hs[2 * i], hi = hs[2 * i + 1];
        acc.x -= v.x * hr - v.y * hi;
        acc.y -= v.x * hi + v.y * hr;
    }
    *w = acc;
}

// ||w||, v_{j+1} = w / ||w||, then the Givens update of column j of H.
__global__ __launch_bounds__(256)
void k_arnoldi_finalize(const Job *__restrict__ jobs, SlotsDev sl, int P, StepStatus *__restrict__ st) {
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
    if (t != 0) return;
    double *col = sl.H + jb.slot * sl.hstride + 2 * hoff(j);
    double *cs = sl.cs + (int64_t)jb.slot * sl.m;
    double *sn = sl.sn + (int64_t)jb.slot * sl.m * 2;
    double *g = sl.g + (int64_t)jb.slot * (sl.m + 1) * 2;
    col[2 * (j + 1)] = hn;
    col[2 * (j + 1) + 1] = 0.0;
    // previous rotations G_i = [[c, s], [-conj(s), c]] on rows (i, i+1)
    for (int i = 0; i < j; ++i) {
        const double c = cs[i], sr = sn[2 * i], si = sn[2 * i + 1];
        const double ar = col[2 * i], ai = col[2 * i + 1];
        const double br = col[2 * i + 2], bi = col[2 * i + 3];
        col[2 * i] = c * ar + (sr * br - si * bi);
        col[2 * i + 1] = c * ai + (sr * bi + si * br);
        col[2 * i + 2] = -(sr * ar + si * ai) + c * br;
        col[2 * i + 3] = -(sr * ai - si * ar) + c * bi;
    }
    // new rotation zeroing h_{j+1,j} (real, >= 0)
    const double ar = col[2 * j], ai = col[2 * j + 1];
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
    cs[j] = c; sn[2 * j] = sr; sn[2 * j + 1] = si;
    col[2 * j] = rr; col[2 * j + 1] = ri;
    col[2 * (j + 1)] = 0.0; col[2 * (j + 1) + 1] = 0.0;
    const double gr = g[2 * j], gi = g[2 * j + 1];
    // g_{j+1} = -conj(s) g_j, g_j = c g_j
    g[2 * (j + 1)] = -(sr * gr + si * gi);
    g[2 * (j + 1) + 1] = -(sr * gi - si * gr);
    g[2 * j] = c * gr;
    g[2 * j + 1] = c * gi;
    st[q].value = sqrt(g[2 * (j + 1)] * g[2 * (j + 1)] + g[2 * (j + 1) + 1] * g[2 * (j + 1) + 1]);
    st[q].hnext = hn;
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
// y = R^{-1} g over the cycle length L = jobs[q].j (R = rotated Hessenberg).
__global__ __launch_bounds__(256)
void k_trisolve(const Job *__restrict__ jobs, SlotsDev sl) {
    extern __shared__ double gs[];
    __shared__ double yi[2];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
    const int L = jb.j;
    const double *H = sl.H + jb.slot * sl.hstride;
    const double *g = sl.g + (int64_t)jb.slot * (sl.m + 1) * 2;
    double *y = sl.y + (int64_t)jb.slot * sl.m * 2;
    for (int i = t; i < 2 * L; i += 256) gs[i] = g[i];
    for (int i = L - 1; i >= 0; --i) {
        __syncthreads();
        if (t == 0) {
            const double *col = H + 2 * hoff(i);
            const double dr = col[2 * i], di = col[2 * i + 1];
            const double den = dr * dr + di * di;
            const double nr = gs[2 * i], ni = gs[2 * i + 1];
            double vr = 0.0, vi = 0.0;
            if (den > 0.0) {
                vr = (nr * dr + ni * di) / den;
                vi = (ni * dr - nr * di) / den;
            }
            yi[0] = vr; yi[1] = vi;
            y[2 * i] = vr; y[2 * i + 1] = vi;
        }
        __syncthreads();
        const double vr = yi[0], vi = yi[1];
        const double *col = H + 2 * hoff(i);
        for (int k = t; k < i; k += 256) {
            const double rr = col[2 * k], ri = col[2 * k + 1];
            gs[2 * k] -= rr * vr - ri * vi;
            gs[2 * k + 1] -= rr * vi + ri * vr;
        }
    }
}

// x += sum_{i<L} v_i y_i
__global__ __launch_bounds__(256)
void k_xupdate(const Job *__restrict__ jobs, SlotsDev sl, int P) {
    extern __shared__ double ys[];
    const int q = blockIdx.y, t = threadIdx.x;
    const Job jb = jobs[q];
    const int L = jb.j;
    const double *y = sl.y + (int64_t)jb.slot * sl.m * 2;
    for (int i = t; i < 2 * L; i += 256) ys[i] = y[i];
    __syncthreads();
    const int mu = blockIdx.x * 256 + t;
    if (mu >= P) return;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    const double *V = sl.V + jb.slot * sl.vstride;
    double2 *x = reinterpret_cast<double2 *>(sl.x + jb.slot * vlen) + mu;
    double2 acc = *x;
    for (int i = 0; i < L; ++i) {
        const double2 v = reinterpret_cast<const double2 *>(V + (int64_t)i * vlen)[mu];
        const double r = ys[2 * i], m = ys[2 * i + 1];
        acc.x += v.x * r - v.y * m;
        acc.y += v.x * m + v.y * r;
    }
    *x = acc;
}

void launch_update_x(Tracer *t, hipStream_t s, const Job *jobs, int n, int jmax,
                     const SlotsDev &sl, int P, double sum_L) {
    const size_t shm = (size_t)(jmax > 0 ? jmax : 1) * 2 * sizeof(double);
    trace_begin(t, "trisolve", s);
    hipLaunchKernelGGL(k_trisolve, dim3(n), dim3(256), shm, s, jobs, sl);
    trace_end(t, s);
    trace_begin(t, "x_update", s);
    hipLaunchKernelGGL(k_xupdate, dim3((P + 255) / 256, n), dim3(256), shm, s, jobs, sl, P);
    trace_end(t, s, 8.0 * P * sum_L, 16.0 * P * (sum_L + 2.0 * n));
}

// ------------------------------------------------------------ polarizability
// alpha[point][k] = -d_k . x  (bilinear, eq. eqpolarizability with alpha = -P);
// jobs[q].j holds the point index.
__global__ __launch_bounds__(256)
void k_alpha(const Job *__restrict__ jobs, SlotsDev sl, const double *__restrict__ drives,
             int n_drive, int P_pad, int P, double *__restrict__ out) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const Job jb = jobs[q];
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
            out[((int64_t)jb.j * n_drive + k) * 2] = -re;
            out[((int64_t)jb.j * n_drive + k) * 2 + 1] = -im;
        }
    }
}

void launch_alpha(Tracer *t, hipStream_t s, const Job *jobs, int n, const SlotsDev &sl,
                  const double *drives, int n_drive, int P_pad, int P, const int32_t *out_index,
                  double *alpha_out) {
    (void)out_index;
    trace_begin(t, "alpha", s);
    hipLaunchKernelGGL(k_alpha, dim3(n), dim3(256), 0, s, jobs, sl, drives, n_drive, P_pad, P, alpha_out);
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
