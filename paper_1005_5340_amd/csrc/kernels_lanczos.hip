// Lanczos recursion in transition space and the spectrum read off it.
//
// In the space of (occupied E, virtual F) transitions the response of Sec. 3
// has the pole form (Casida's equations)
//     Om2 = diag(D^2) + S V_t^T f V_t S,  S = diag(sqrt(2 n D)),  c = S V_t^T d,
//     alpha(w) = c^T (Om2 - (w + i eps)^2)^-1 c,
// with D_EF = e_F - e_E, v^{EF} the transition vertices of eq. response-mat
// (V_t: n_prod x T) and f the kernel of eq. sle.  The symmetric Lanczos
// recursion on Om2 started from c gives a tridiagonal T_k from which
// alpha(w) follows at every frequency (a continued fraction) and the poles
// and residues follow from T_k's eigen-decomposition: the economical
// treatment of the frequency axis, with pole positions and strengths, that
// Sec. 8 names as further work.  Om2 is applied matrix-free by the chi0
// operator's own kernels (the back half (b3), (b4), (d), then K, then the
// front half (a), (b1), (b2)); this file holds the recursion's vector work.
//
// A block of nc <= 4 recursions (one per drive) runs together.  The
// recursion's vectors are compact: transition (F, E) is row F * No + E of
// tc rows (No * Nv rounded up to 64, the tail kept at zero), sequence s in
// column s, so the basis passes stream no padding.  The operator's buffer
// `at` keeps its GEMM layout, row F * No_pad + E; the kernels that meet both
// map one row index to the other.  The step index lives in device memory so that
// one step's launch sequence can be replayed from a HIP graph.  Reductions
// are deterministic: fixed-order per-workgroup sums, then one workgroup adds
// the partials in a fixed order.
#include "common.h"

namespace chi0 {

namespace {

__device__ __forceinline__ double lz_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-workgroup sums of NC accumulators into part[blockIdx.x][NC] (256 threads).
template <int NC>
__device__ __forceinline__ void lz_block_part(const double (&acc)[NC], double *part) {
    __shared__ double sh[4][NC];
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const double v = lz_wave_sum(acc[s]);
        if ((t & 63) == 0) sh[t >> 6][s] = v;
    }
    __syncthreads();
    if (t < NC) part[(int64_t)blockIdx.x * NC + t] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
}

// Sum of the nblk partials of sequence s by one 256-thread workgroup (fixed order).
template <int NC>
__device__ __forceinline__ double lz_sum_parts(const double *part, int nblk, int s, double *sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) v += part[(int64_t)b * NC + s];
    v = lz_wave_sum(v);
    const int t = threadIdx.x;
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__device__ __forceinline__ double *lz_vec(const LanczosDev &L, int i) {
    return L.R + (int64_t)(L.ring ? i % 3 : i) * L.n;
}

}  // namespace

// St = sqrt(2 n D), D2t = D^2 on the compact rows (0 on the tail).
__global__ __launch_bounds__(256)
void k_lz_tables(const double *__restrict__ Dlt, int No, int Nv, int nv_pad, int64_t tc, double occ,
                 double *__restrict__ St, double *__restrict__ D2t) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= tc) return;
    double s = 0.0, d2 = 0.0;
    if (idx < (int64_t)No * Nv) {
        const int F = (int)(idx / No), E = (int)(idx % No);
        const double d = Dlt[(int64_t)E * nv_pad + F];
        s = sqrt(2.0 * occ * d);
        d2 = d * d;
    }
    St[idx] = s;
    D2t[idx] = d2;
}

// Row of `at` (GEMM layout) of compact row r < No * Nv.
__device__ __forceinline__ int64_t lz_prow(const LanczosDev &L, int64_t r) {
    return (r / L.no) * L.no_pad + r % L.no;
}

// Start: R[0] = St * at (c = S V_t^T d, the front half already applied to d);
// partial sums of |c|^2.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_start(LanczosDev L) {
    double acc[NC] = {};
    double *q = lz_vec(L, 0);
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < L.t_alg; r += (int64_t)gridDim.x * 256) {
        const double st = L.St[r];
        const int64_t rp = lz_prow(L, r);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const double v = st * L.at[rp * NC + s];
            q[r * NC + s] = v;
            acc[s] += v * v;
        }
    }
    lz_block_part<NC>(acc, L.part);
}

// |c|^2 per sequence; a sequence with c = 0 has length 0.  Resets the step counter.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_start_fin(LanczosDev L, int nblk) {
    __shared__ double sh[4];
    for (int s = 0; s < NC; ++s) {
        const double v = lz_sum_parts<NC>(L.part, nblk, s, sh);
        if (threadIdx.x == 0) {
            L.cn2[s] = v;
            L.len[s] = v > 0.0 ? L.kmax : 0;
        }
    }
    if (threadIdx.x == 0) *L.step = 0;
}

// q *= inv (per sequence) in place on the compact rows, and at = St * q on
// every row of `at` (0 on its padding), one thread per row of `at`.
template <int NC>
__device__ __forceinline__ void lz_normalise_to_at(const LanczosDev &L, double *q, const double (&inv)[NC]) {
    for (int64_t rp = (int64_t)blockIdx.x * 256 + threadIdx.x; rp < L.tp; rp += (int64_t)gridDim.x * 256) {
        const int F = (int)(rp / L.no_pad), E = (int)(rp % L.no_pad);
        if (E < L.no && F < L.nv) {
            const int64_t r = (int64_t)F * L.no + E;
            const double st = L.St[r];
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                const double v = q[r * NC + s] * inv[s];
                q[r * NC + s] = v;
                L.at[rp * NC + s] = st * v;
            }
        } else {
#pragma unroll
            for (int s = 0; s < NC; ++s) L.at[rp * NC + s] = 0.0;
        }
    }
}

// q_0 = c / |c| in place; at = St * q_0 (input of the next operator pass).
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_start_scale(LanczosDev L) {
    double inv[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) inv[s] = L.cn2[s] > 0.0 ? 1.0 / sqrt(L.cn2[s]) : 0.0;
    double *q = lz_vec(L, 0);
    lz_normalise_to_at<NC>(L, q, inv);
}

// Step j, after the operator pass: w = St * at + D2t * q_j (= Om2 q_j) into
// vector j + 1; partial sums of q_j . w.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_combine(LanczosDev L) {
    const int j = *L.step;
    const double *q = lz_vec(L, j);
    double *w = lz_vec(L, j + 1);
    double acc[NC] = {};
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < L.t_alg; r += (int64_t)gridDim.x * 256) {
        const double st = L.St[r], d2 = L.D2t[r];
        const int64_t rp = lz_prow(L, r);
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const double qv = q[r * NC + s];
            const double v = st * L.at[rp * NC + s] + d2 * qv;
            w[r * NC + s] = v;
            acc[s] += qv * v;
        }
    }
    lz_block_part<NC>(acc, L.part);
}

// a_j = q_j . w; advances the step counter (later kernels of the step read j = step - 1).
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_alpha(LanczosDev L, int nblk) {
    __shared__ double sh[4];
    const int j = *L.step;
    for (int s = 0; s < NC; ++s) {
        const double v = lz_sum_parts<NC>(L.part, nblk, s, sh);
        if (threadIdx.x == 0) L.a[(int64_t)j * NC + s] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) *L.step = j + 1;
}

// w -= a_j q_j + b_{j-1} q_{j-1}; partial sums of |w|^2.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_axpy(LanczosDev L) {
    const int j = *L.step - 1;
    const double *q = lz_vec(L, j);
    const double *qm = lz_vec(L, j > 0 ? j - 1 : 0);
    double *w = lz_vec(L, j + 1);
    double aj[NC], bm[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        aj[s] = L.a[(int64_t)j * NC + s];
        bm[s] = j > 0 ? L.b[(int64_t)(j - 1) * NC + s] : 0.0;
    }
    double acc[NC] = {};
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < L.tc; r += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            const double v = w[r * NC + s] - aj[s] * q[r * NC + s] - bm[s] * qm[r * NC + s];
            w[r * NC + s] = v;
            acc[s] += v * v;
        }
    }
    lz_block_part<NC>(acc, L.part);
}

// b_j = |w|.  A sequence ends (length j + 1, b_j = 0 and every later
// coefficient 0) when b_j <= 1e-12 (|a_j| + b_{j-1}): an invariant subspace.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_beta(LanczosDev L, int nblk, int gated) {
    if (gated && L.flag && !L.flag[0]) return;   // no pass: b_j of the head stands
    __shared__ double sh[4];
    const int j = *L.step - 1;
    for (int s = 0; s < NC; ++s) {
        const double v = lz_sum_parts<NC>(L.part, nblk, s, sh);
        if (threadIdx.x == 0) {
            const double bj = sqrt(v);
            const double aj = L.a[(int64_t)j * NC + s];
            const double bm = j > 0 ? L.b[(int64_t)(j - 1) * NC + s] : 0.0;
            const bool ended = L.len[s] <= j || !(bj > 1e-12 * (fabs(aj) + bm));
            if (ended && L.len[s] > j) L.len[s] = j + 1;
            L.b[(int64_t)j * NC + s] = ended ? 0.0 : bj;
        }
    }
}

// q_{j+1} = w / b_j in place (0 for an ended sequence); at = St * q_{j+1}.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_scale(LanczosDev L) {
    const int j = *L.step - 1;
    double *w = lz_vec(L, j + 1);
    double inv[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const double bj = L.b[(int64_t)j * NC + s];
        inv[s] = bj > 0.0 ? 1.0 / bj : 0.0;
    }
    lz_normalise_to_at<NC>(L, w, inv);
}

// Full reorthogonalisation: classical Gram-Schmidt passes against q_0..q_j.
// The basis is streamed once per kernel and is far larger than the caches, so
// its loads are non-temporal 16-byte loads; w (one vector) stays in L2.  A
// vector of n = tp * NC doubles is read as n / 2 pairs (tp is even); pair p
// holds the elements of sequences (2p) % NC and (2p + 1) % NC.  For NC = 1, 2
// and 4 a thread's pairs all hold the same two sequences (its pairs are 256
// apart, and 512 elements is a multiple of NC); NC = 3 reads single elements.
typedef double lz_dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ lz_dbl2 lz_ld2nt(const double *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const lz_dbl2 *>(p));
}
__device__ __forceinline__ double lz_ldnt(const double *p) { return __builtin_nontemporal_load(p); }

// h[i][s] = q_i . w over pairs [rs * chunk, ...), per (split rs, vector i).
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_dots(LanczosDev L, int nq, int nsplit, double *part2) {
    if (L.flag && !L.flag[0]) return;   // partial reorthogonalisation: no pass this step
    const int i = blockIdx.y, rs = blockIdx.x;
    const int j = *L.step - 1;
    const double *q = lz_vec(L, i);
    const double *w = lz_vec(L, j + 1);
    double acc[NC] = {};
    if (NC != 3) {
        const int64_t np = L.n / 2, chunk = ((np + nsplit - 1) / nsplit + 255) / 256 * 256;
        const int64_t p0 = rs * chunk, p1 = min(np, p0 + chunk);
        const int sa = (int)((2 * (p0 + threadIdx.x)) % NC), sb = (sa + 1) % NC;
        double x = 0.0, y = 0.0;
#pragma unroll 4
        for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
            const lz_dbl2 qv = lz_ld2nt(q + 2 * p);
            const double2 wv = *reinterpret_cast<const double2 *>(w + 2 * p);
            x += qv.x * wv.x;
            y += qv.y * wv.y;
        }
#pragma unroll
        for (int s = 0; s < NC; ++s) acc[s] = (s == sa ? x : 0.0) + (s == sb ? y : 0.0);
    } else {
        const int64_t chunk = (L.tc + nsplit - 1) / nsplit;
        const int64_t r0 = rs * chunk, r1 = min(L.tc, r0 + chunk);
#pragma unroll 4
        for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
#pragma unroll
            for (int s = 0; s < NC; ++s) acc[s] += lz_ldnt(q + r * NC + s) * w[r * NC + s];
        }
    }
    __shared__ double sh[4][NC];
    const int t = threadIdx.x;
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        const double v = lz_wave_sum(acc[s]);
        if ((t & 63) == 0) sh[t >> 6][s] = v;
    }
    __syncthreads();
    if (t < NC && i < nq)
        part2[((int64_t)i * nsplit + rs) * NC + t] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
}

template <int NC>
__global__ __launch_bounds__(256)
void k_lz_dots_fin(const double *part2, int nq, int nsplit, double *h, const int *flag) {
    if (flag && !flag[0]) return;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)nq * NC) return;
    const int i = (int)(idx / NC), s = (int)(idx % NC);
    double v = 0.0;
    for (int rs = 0; rs < nsplit; ++rs) v += part2[((int64_t)i * nsplit + rs) * NC + s];
    h[idx] = v;
}

// part3[g][e] = sum over the vectors i of group g (a contiguous range) of
// q_i[e] h[i][seq(e)]; workgroup (block of pairs, group): one pair per thread
// (NC = 3: one row of three per thread).
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_update_part(LanczosDev L, int nq, int ngroup, const double *__restrict__ h, double *__restrict__ part3) {
    if (L.flag && !L.flag[0]) return;
    const int g = blockIdx.y;
    const int per = (nq + ngroup - 1) / ngroup;
    const int i0 = g * per, i1 = min(nq, i0 + per);
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (NC != 3) {
        if (u >= L.n / 2) return;
        const int sa = (int)((2 * u) % NC), sb = (sa + 1) % NC;
        double x = 0.0, y = 0.0;
        int i = i0;
        for (; i + 8 <= i1; i += 8) {
            lz_dbl2 qv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) qv[k] = lz_ld2nt(lz_vec(L, i + k) + 2 * u);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                x += qv[k].x * h[(int64_t)(i + k) * NC + sa];
                y += qv[k].y * h[(int64_t)(i + k) * NC + sb];
            }
        }
        for (; i < i1; ++i) {
            const lz_dbl2 qv = lz_ld2nt(lz_vec(L, i) + 2 * u);
            x += qv.x * h[(int64_t)i * NC + sa];
            y += qv.y * h[(int64_t)i * NC + sb];
        }
        *reinterpret_cast<double2 *>(part3 + (int64_t)g * L.n + 2 * u) = make_double2(x, y);
    } else {
        const int64_t r = u;
        if (r >= L.tc) return;
        double acc[NC] = {};
        for (int i = i0; i < i1; ++i)
#pragma unroll
            for (int s = 0; s < NC; ++s) acc[s] += lz_ldnt(lz_vec(L, i) + r * NC + s) * h[(int64_t)i * NC + s];
#pragma unroll
        for (int s = 0; s < NC; ++s) part3[(int64_t)g * L.n + r * NC + s] = acc[s];
    }
}

// w -= sum_g part3[g] (groups in order); partial sums of |w|^2.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_update_fin(LanczosDev L, int ngroup, const double *__restrict__ part3) {
    if (L.flag && !L.flag[0]) return;
    const int j = *L.step - 1;
    double *w = lz_vec(L, j + 1);
    double acc[NC] = {};
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < L.tc; r += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int s = 0; s < NC; ++s) {
            double sub = 0.0;
            for (int g = 0; g < ngroup; ++g) sub += part3[(int64_t)g * L.n + r * NC + s];
            const double v = w[r * NC + s] - sub;
            w[r * NC + s] = v;
            acc[s] += v * v;
        }
    }
    lz_block_part<NC>(acc, L.part);
}

// alpha_k(w) = |c|^2 / g_0 with g_{k-1} = a_{k-1} - z, g_i = a_i - z - b_i^2 / g_{i+1},
// z = (w + i eps)^2: the continued fraction of |c|^2 e_1^T (T_k - z)^-1 e_1.
// One thread per (frequency, sequence); k = min(kuse, len[s]).
__global__ __launch_bounds__(256)
void k_lz_cfrac(const double *__restrict__ a, const double *__restrict__ b, int nc, int kuse,
                const int *__restrict__ len, const double *__restrict__ cn2, const double *__restrict__ omega,
                int n_omega, double eps, double *__restrict__ out) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n_omega * nc) return;
    const int wi = idx / nc, s = idx % nc;
    const int k = min(kuse, len[s]);
    const double w = omega[wi];
    const double zr = w * w - eps * eps, zi = 2.0 * w * eps;
    double gr = 0.0, gi = 0.0;
    if (k > 0) {
        gr = a[(int64_t)(k - 1) * nc + s] - zr;
        gi = -zi;
        for (int i = k - 2; i >= 0; --i) {
            const double bb = b[(int64_t)i * nc + s];
            const double m = gr * gr + gi * gi;           // -b^2 / g = -b^2 conj(g) / |g|^2
            const double f = bb * bb / m;
            gr = a[(int64_t)i * nc + s] - zr - f * gr;
            gi = -zi + f * gi;
        }
    }
    double re = 0.0, im = 0.0;   // an empty recursion (c = 0) gives alpha = 0
    if (k > 0) {
        const double m = gr * gr + gi * gi;
        re = cn2[s] * gr / m;
        im = -cn2[s] * gi / m;
    }
    out[2 * (int64_t)idx] = re;
    out[2 * (int64_t)idx + 1] = im;
}

// Partial reorthogonalisation (Simon's omega recurrence), one workgroup: from a_j,
// the head's b_j and the earlier coefficients, the estimates of q_{j+1} . q_i for
// i < j; the pass runs when one exceeds sqrt(eps) (or the previous step ran it on
// its own estimate: the next vector is reorthogonalised too), and the estimates of
// a reorthogonalised vector restart at eps.  Same arithmetic as the recurrence
// written out sequentially; the maximum does not depend on the order.
constexpr int LZ_OMEGA_THREADS = 1024;
__global__ __launch_bounds__(LZ_OMEGA_THREADS)
void k_lz_omega(LanczosDev L, int j) {
    const int nc = L.nc, t = threadIdx.x;
    const int64_t rl = (int64_t)L.kmax + 2;
    const double ueps = 2.220446049250313e-16, thresh = 1.4901161193847656e-08;   // sqrt(eps)
    double *const Wr = L.omega;
    __shared__ double sh[LZ_OMEGA_THREADS / 64];
    __shared__ int need_s;
    if (t == 0) need_s = L.flag[1];
    __syncthreads();
    for (int s = 0; s < nc; ++s) {
        const double *wc = Wr + ((int64_t)(j % 3) * nc + s) * rl;         // row j
        const double *wp = Wr + ((int64_t)((j + 2) % 3) * nc + s) * rl;   // row j - 1
        double *wn = Wr + ((int64_t)((j + 1) % 3) * nc + s) * rl;         // row j + 1
        const double aj = L.a[(int64_t)j * nc + s], bj = L.b[(int64_t)j * nc + s];
        const double bm = j > 0 ? L.b[(int64_t)(j - 1) * nc + s] : 0.0;
        if (!(bj > 0.0)) continue;   // ended sequence (uniform across the workgroup)
        const double an = fmax(L.anorm[s], fabs(aj) + bj + bm);
        double mx = 0.0;
        for (int i = t; i < j; i += LZ_OMEGA_THREADS) {
            const double bi = L.b[(int64_t)i * nc + s];
            double tv = bi * wc[i + 1] + (L.a[(int64_t)i * nc + s] - aj) * wc[i] - bm * wp[i];
            if (i > 0) tv += L.b[(int64_t)(i - 1) * nc + s] * wc[i - 1];
            const double v = (tv + (tv >= 0.0 ? 1.0 : -1.0) * 2.0 * ueps * an) / bj;
            wn[i] = v;
            mx = fmax(mx, fabs(v));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        __syncthreads();
        if ((t & 63) == 0) sh[t >> 6] = mx;
        __syncthreads();
        if (t == 0) {
            double m = 0.0;
            for (int w = 0; w < LZ_OMEGA_THREADS / 64; ++w) m = fmax(m, sh[w]);
            if (m > thresh) need_s = 1;
            wn[j] = ueps * an / bj;
            wn[j + 1] = 1.0;
            L.anorm[s] = an;
        }
        __syncthreads();
    }
    const int need = need_s;
    if (need)   // the new vector is reorthogonalised: its estimates restart at eps
        for (int s = 0; s < nc; ++s) {
            double *wn = Wr + ((int64_t)((j + 1) % 3) * nc + s) * rl;
            for (int i = t; i <= j; i += LZ_OMEGA_THREADS) wn[i] = ueps;
        }
    if (t == 0) {
        L.flag[0] = need;
        L.flag[1] = need ? !L.flag[1] : 0;
    }
}

// ------------------------------------------------------- solutions of eq. sle
// x_i(w) = -B (Om2 - z)^-1 c_i with B = V_t S, approximated in the Krylov basis
// as -B Q_k y, y = |c_i| (T_k - z)^-1 e_1, z = (w + i eps)^2.  LZ_XW frequencies
// per pass, LZ_XW / NC... columns: column m = w * NC + s of sequence s.

// y for every (frequency w, sequence s) of a pass: T_k - z is complex symmetric
// tridiagonal with Im z > 0 for w > 0, so elimination without pivoting keeps
// every pivot's imaginary part <= -Im z (never zero).  Forward pivots and
// right-hand side in dw, then back substitution into Y[i][m] (complex), zero for
// i >= len[s] up to kuse.
__global__ __launch_bounds__(64)
void k_lz_tsolve(const double *__restrict__ a, const double *__restrict__ b, int nc, int kuse,
                 const int *__restrict__ len, const double *__restrict__ cn2, const double *__restrict__ omega,
                 int nw, double eps, double *__restrict__ dw, double *__restrict__ Y) {
    const int m = blockIdx.x * 64 + threadIdx.x, ncol = nw * nc;
    if (m >= ncol) return;
    const int w = m / nc, s = m % nc;
    const int k = min(kuse, len[s]);
    const double om = omega[w];
    const double zr = om * om - eps * eps, zi = 2.0 * om * eps;
    // dw[i] = (d_r, d_i, g_r, g_i) of row i
    double dr = 0.0, di = 0.0, gr = 0.0, gi = 0.0;
    for (int i = 0; i < k; ++i) {
        const double ai = a[(int64_t)i * nc + s];
        if (i == 0) {
            dr = ai - zr;
            di = -zi;
            gr = sqrt(cn2[s]);
            gi = 0.0;
        } else {
            const double bb = b[(int64_t)(i - 1) * nc + s];
            // l = bb / d_{i-1};  d_i = a_i - z - l bb;  g_i = -l g_{i-1}
            const double m2 = dr * dr + di * di;
            const double lr = bb * dr / m2, li = -bb * di / m2;
            const double ngr = -(lr * gr - li * gi), ngi = -(lr * gi + li * gr);
            dr = ai - zr - lr * bb;
            di = -zi - li * bb;
            gr = ngr;
            gi = ngi;
        }
        double *p = dw + ((int64_t)i * ncol + m) * 4;
        p[0] = dr;
        p[1] = di;
        p[2] = gr;
        p[3] = gi;
    }
    double yr = 0.0, yi = 0.0;   // y_{i+1}
    for (int i = kuse - 1; i >= 0; --i) {
        double vr = 0.0, vi = 0.0;
        if (i < k) {
            const double *p = dw + ((int64_t)i * ncol + m) * 4;
            const double bb = i + 1 < k ? b[(int64_t)i * nc + s] : 0.0;
            const double tr = p[2] - bb * yr, ti = p[3] - bb * yi;   // (g_i - b_i y_{i+1}) / d_i
            const double m2 = p[0] * p[0] + p[1] * p[1];
            vr = (tr * p[0] + ti * p[1]) / m2;
            vi = (ti * p[0] - tr * p[1]) / m2;
        }
        Y[((int64_t)i * ncol + m) * 2] = vr;
        Y[((int64_t)i * ncol + m) * 2 + 1] = vi;
        yr = vr;
        yi = vi;
    }
}

// at[rp][2m + re/im] = St[r] * sum_{i < kuse} q_i[r][s] Y[i][m] for the W * NC columns
// of a pass (0 on the padding of `at`): the back half then gives B Q_k y.
template <int NC>
__global__ __launch_bounds__(256)
void k_lz_expand(LanczosDev L, int kuse, const double *__restrict__ Y, double *__restrict__ at) {
    constexpr int W = LZ_XCOL / NC, M = W * NC;
    const int64_t rp = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (rp >= L.tp) return;
    const int F = (int)(rp / L.no_pad), E = (int)(rp % L.no_pad);
    double acc[M][2];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m][0] = acc[m][1] = 0.0;
    if (E < L.no && F < L.nv) {
        const int64_t r = (int64_t)F * L.no + E;
        for (int i = 0; i < kuse; ++i) {
            double qv[NC];
#pragma unroll
            for (int s = 0; s < NC; ++s) qv[s] = lz_ldnt(lz_vec(L, i) + r * NC + s);
            const double *y = Y + (int64_t)i * M * 2;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                acc[m][0] += qv[m % NC] * y[2 * m];
                acc[m][1] += qv[m % NC] * y[2 * m + 1];
            }
        }
        const double st = L.St[r];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            acc[m][0] *= st;
            acc[m][1] *= st;
        }
    }
    double *o = at + rp * (2 * M);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        o[2 * m] = acc[m][0];
        o[2 * m + 1] = acc[m][1];
    }
}

// From Yb = B Q_k y [P_pad][2M] (column 2m + re/im): x rows out[w][s][mu] = -Yb[mu][m]
// (complex) for the nw valid frequencies, and alpha[w][k][i] = -d_k . x_i = d_k . Yb[:, m(w, i)].
__global__ __launch_bounds__(256)
void k_lz_x_rows(const double *__restrict__ Yb, int M, int nc, int nw, int P, double *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)nw * nc * P) return;
    const int m = (int)(idx / P), mu = (int)(idx % P);
    out[2 * idx] = -Yb[(int64_t)mu * 2 * M + 2 * m];
    out[2 * idx + 1] = -Yb[(int64_t)mu * 2 * M + 2 * m + 1];
}

__global__ __launch_bounds__(256)
void k_lz_alpha_x(const double *__restrict__ Yb, int M, int nc, int P, const double *__restrict__ drives,
                  double *__restrict__ alpha) {
    // workgroup (w, k, i): drives [nc][P] host order
    const int w = blockIdx.x, k = blockIdx.y, i = blockIdx.z;
    const int m = w * nc + i;
    double sr = 0.0, si = 0.0;
    for (int mu = threadIdx.x; mu < P; mu += 256) {
        const double dk = drives[(int64_t)k * P + mu];
        sr += dk * Yb[(int64_t)mu * 2 * M + 2 * m];
        si += dk * Yb[(int64_t)mu * 2 * M + 2 * m + 1];
    }
    __shared__ double sh[2][4];
    sr = lz_wave_sum(sr);
    si = lz_wave_sum(si);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = sr;
        sh[1][threadIdx.x >> 6] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t o = (((int64_t)w * nc + k) * nc + i) * 2;
        alpha[o] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        alpha[o + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// ------------------------------------------------------------------ launches
namespace {
int lz_blocks(const LanczosDev &L) {
    int64_t b = (std::max(L.tp, L.tc) + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), LZ_BLOCKS);
}
}  // namespace

#define LZ_NC_SWITCH(nc, CALL) \
    switch (nc) {              \
    case 1: CALL(1); break;    \
    case 2: CALL(2); break;    \
    case 3: CALL(3); break;    \
    default: CALL(4); break;   \
    }

void launch_lz_tables(hipStream_t s, const double *Dlt, int No, int Nv, int nv_pad, int64_t tc, double occ,
                      double *St, double *D2t) {
    hipLaunchKernelGGL(k_lz_tables, dim3((unsigned)((tc + 255) / 256)), dim3(256), 0, s, Dlt, No, Nv, nv_pad, tc,
                       occ, St, D2t);
}

void launch_lz_start(Tracer *t, hipStream_t s, const LanczosDev &L) {
    const int g = lz_blocks(L);
    trace_begin(t, "lanczos_start", s);
#define C(N)                                                                        \
    hipLaunchKernelGGL(k_lz_start<N>, dim3(g), dim3(256), 0, s, L);                 \
    hipLaunchKernelGGL(k_lz_start_fin<N>, dim3(1), dim3(256), 0, s, L, g);          \
    hipLaunchKernelGGL(k_lz_start_scale<N>, dim3(g), dim3(256), 0, s, L);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s, 0.0, 8.0 * (double)L.t_alg * L.nc * 4);
}

namespace {
// combine (w = Om2 q_j), a_j, the three-term update
void lz_head(Tracer *t, hipStream_t s, const LanczosDev &L, int g, double ta, double vb) {
    trace_begin(t, "lanczos_combine", s);
#define C(N)                                                                   \
    hipLaunchKernelGGL(k_lz_combine<N>, dim3(g), dim3(256), 0, s, L);          \
    hipLaunchKernelGGL(k_lz_alpha<N>, dim3(1), dim3(256), 0, s, L, g);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s, 4.0 * ta, 3.0 * vb + 16.0 * L.t_alg);
    trace_begin(t, "lanczos_axpy", s);
#define C(N) hipLaunchKernelGGL(k_lz_axpy<N>, dim3(g), dim3(256), 0, s, L);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s, 6.0 * ta, 4.0 * vb);
}

// npass classical Gram-Schmidt passes of w against q_0..q_j (j known on the host)
void lz_passes(Tracer *t, hipStream_t s, const LanczosDev &L, int j, int npass, int g, double ta, double vb,
               double *part2, double *h, double *part3) {
    const int nq = j + 1;
    const int nsplit = std::max(1, std::min(64, 2048 / nq));
    const unsigned rblocks = (unsigned)(((L.nc == 3 ? L.tc : L.n / 2) + 255) / 256);
    const int ngroup = std::max(1, std::min(LZ_GROUPS, nq / 64));
    for (int pass = 0; pass < npass; ++pass) {
        trace_begin(t, "lanczos_reorth_dots", s);
#define C(N)                                                                                                  \
    hipLaunchKernelGGL(k_lz_dots<N>, dim3(nsplit, nq), dim3(256), 0, s, L, nq, nsplit, part2);                \
    hipLaunchKernelGGL(k_lz_dots_fin<N>, dim3((unsigned)((nq * N + 255) / 256)), dim3(256), 0, s, part2, nq, \
                       nsplit, h, L.flag);
        LZ_NC_SWITCH(L.nc, C)
#undef C
        trace_end(t, s, 2.0 * ta * nq, vb * (nq + 1));
        trace_begin(t, "lanczos_reorth_update", s);
#define C(N)                                                                                                   \
    hipLaunchKernelGGL(k_lz_update_part<N>, dim3(rblocks, ngroup), dim3(256), 0, s, L, nq, ngroup, h, part3); \
    hipLaunchKernelGGL(k_lz_update_fin<N>, dim3(g), dim3(256), 0, s, L, ngroup, part3);
        LZ_NC_SWITCH(L.nc, C)
#undef C
        trace_end(t, s, 2.0 * ta * nq, vb * (nq + 2));
    }
}

void lz_beta(Tracer *t, hipStream_t s, const LanczosDev &L, int g, int gated = 0) {
    trace_begin(t, "lanczos_beta", s);
#define C(N) hipLaunchKernelGGL(k_lz_beta<N>, dim3(1), dim3(256), 0, s, L, g, gated);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s);
}

void lz_scale(Tracer *t, hipStream_t s, const LanczosDev &L, int g, double ta, double vb) {
    trace_begin(t, "lanczos_scale", s);
#define C(N) hipLaunchKernelGGL(k_lz_scale<N>, dim3(g), dim3(256), 0, s, L);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s, 2.0 * ta, 3.0 * vb + 8.0 * L.t_alg);
}
}  // namespace

void launch_lz_step(Tracer *t, hipStream_t s, const LanczosDev &L, int j, double *part2, double *h,
                    double *part3) {
    const int g = lz_blocks(L);
    // algorithmic work on unpadded transitions: one vector of the block is 8 T nc bytes
    const double ta = (double)L.t_alg * L.nc, vb = 8.0 * ta;
    lz_head(t, s, L, g, ta, vb);
    if (!L.ring) lz_passes(t, s, L, j, L.passes, g, ta, vb, part2, h, part3);
    lz_beta(t, s, L, g);
    lz_scale(t, s, L, g, ta, vb);
}

// head of a step with partial reorthogonalisation: the three-term update, b_j and
// the device-side decision (flag[0]) on the pass
void launch_lz_step_head(Tracer *t, hipStream_t s, const LanczosDev &L, int j) {
    const int g = lz_blocks(L);
    const double ta = (double)L.t_alg * L.nc, vb = 8.0 * ta;
    lz_head(t, s, L, g, ta, vb);
    lz_beta(t, s, L, g);
    trace_begin(t, "lanczos_omega", s);
    hipLaunchKernelGGL(k_lz_omega, dim3(1), dim3(LZ_OMEGA_THREADS), 0, s, L, j);
    trace_end(t, s);
}

// a whole step with partial reorthogonalisation, no host decision: the pass
// kernels and the second b_j are launched every step and return at once when
// the flag is clear
void launch_lz_step_partial(Tracer *t, hipStream_t s, const LanczosDev &L, int j, double *part2, double *h,
                            double *part3) {
    const int g = lz_blocks(L);
    const double ta = (double)L.t_alg * L.nc, vb = 8.0 * ta;
    launch_lz_step_head(t, s, L, j);
    lz_passes(t, s, L, j, 1, g, ta, vb, part2, h, part3);
    lz_beta(t, s, L, g, 1);
    lz_scale(t, s, L, g, ta, vb);
}

void launch_lz_step_tail(Tracer *t, hipStream_t s, const LanczosDev &L, int j, int npass, double *part2, double *h,
                         double *part3) {
    const int g = lz_blocks(L);
    const double ta = (double)L.t_alg * L.nc, vb = 8.0 * ta;
    if (npass > 0) {
        lz_passes(t, s, L, j, npass, g, ta, vb, part2, h, part3);
        lz_beta(t, s, L, g);
    }
    lz_scale(t, s, L, g, ta, vb);
}

void launch_lz_solution_cols(Tracer *t, hipStream_t s, const LanczosDev &L, int kuse, const int *len,
                             const double *omega, int nw, double eps, double *dw, double *Y, double *at) {
    const int W = LZ_XCOL / L.nc, M = W * L.nc;
    trace_begin(t, "lanczos_solution", s);
    hipLaunchKernelGGL(k_lz_tsolve, dim3((M + 63) / 64), dim3(64), 0, s, L.a, L.b, L.nc, kuse, len, L.cn2, omega,
                       W, eps, dw, Y);
    const unsigned g = (unsigned)((L.tp + 255) / 256);
#define C(N) hipLaunchKernelGGL(k_lz_expand<N>, dim3(g), dim3(256), 0, s, L, kuse, Y, at);
    LZ_NC_SWITCH(L.nc, C)
#undef C
    trace_end(t, s, 4.0 * (double)L.t_alg * M * kuse, 8.0 * (double)L.t_alg * L.nc * kuse);
    (void)nw;
}

void launch_lz_solution_out(hipStream_t s, const double *Yb, int nc, int nw, int P, const double *drives,
                            double *x_rows, double *alpha) {
    const int M = (LZ_XCOL / nc) * nc;
    const int64_t n = (int64_t)nw * nc * P;
    if (x_rows && n > 0)
        hipLaunchKernelGGL(k_lz_x_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Yb, M, nc, nw, P,
                           x_rows);
    if (alpha && nw > 0)
        hipLaunchKernelGGL(k_lz_alpha_x, dim3(nw, nc, nc), dim3(256), 0, s, Yb, M, nc, P, drives, alpha);
}

void launch_lz_cfrac(hipStream_t s, const double *a, const double *b, int nc, int kuse, const int *len,
                     const double *cn2, const double *omega, int n_omega, double eps, double *out) {
    const int n = n_omega * nc;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_lz_cfrac, dim3((n + 255) / 256), dim3(256), 0, s, a, b, nc, kuse, len, cn2, omega,
                       n_omega, eps, out);
}

}  // namespace chi0
