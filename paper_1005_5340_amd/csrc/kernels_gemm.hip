// FP64 MFMA kernels of the orbital transforms (Sec. 4.2, Table t:flops steps
// 2-5) and the kernel matrix-vector product (Sec. 4.1).
//
// All matrix-core work uses v_mfma_f64_16x16x4f64 on 64-lane wavefronts.
// Operand layout of one 16x16x4 step (lane l = 0..63):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[4*r + l/16][l % 16] in element r = 0..3
//                (rows interleaved by 4; checked on gfx950 with a lane probe)
#include "common.h"

namespace chi0 {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Workgroup id -> tile id such that each of the 8 XCDs (which receive
// consecutive workgroup ids round robin) works on one contiguous range of
// tiles; tiles that share an operand strip then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int wid, int n) {
    const int q = n / 8, r = n % 8;
    const int x = wid % 8, local = wid / 8;
    return x * q + (x < r ? x : r) + local;
}

// ------------------------------------------------------------------ dense GEMM
// C[M x N] = A[M x K] B[K x N], row-major, M % BM == 0, K % 16 == 0, N masked.
// Optional epilogue (b2)+(c): C column n <-> (E, j) with E = n / ncp,
// j = n % ncp; columns 2r and 2r+1 hold Re and Im of RHS r; row = virtual F.
struct LorentzArgs {
    const double *Dlt;   // [No_pad][Nv_pad]
    const double *omega; // [ncp/2]
    int nv_pad;
    int ncp;
    double eps;
    double occ;
};

template <int BM, int BN, int WM, int WN, bool LORENTZ>
__global__ __launch_bounds__(WM * WN * 64)
void k_dgemm(int M, int N, int K, const double *__restrict__ A, int lda,
             const double *__restrict__ B, int ldb, double *__restrict__ C, int ldc,
             int m_fastest, LorentzArgs la) {
    constexpr int BK = 16;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 16;
    constexpr int TN = BN / WN / 16;
    constexpr int APT = BM * BK / NT;   // A doubles per thread per tile
    constexpr int BPT = BK * BN / NT;   // B doubles per thread per tile
    static_assert(APT == 4 && BPT == 4, "tile shape must give 4 doubles per thread");
    __shared__ double As[2][BK][BM + 1];
    __shared__ double Bs[2][BK][BN];

    const int ntm = M / BM, ntn = (N + BN - 1) / BN;
    const int tile = xcd_remap(blockIdx.x, ntm * ntn);
    const int tm = m_fastest ? tile % ntm : tile / ntn;
    const int tn = m_fastest ? tile / ntm : tile % ntn;
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;

    // global -> register mapping
    const int a_row = t / 4, a_k = (t % 4) * 4;        // BM rows x 16 k
    const int b_k = t / (BN / 4), b_n = (t % (BN / 4)) * 4;
    const double *Ap = A + (int64_t)(m0 + a_row) * lda + a_k;
    const double *Bp = B + (int64_t)b_k * ldb + n0 + b_n;
    const bool b_full = (n0 + b_n + 3) < N;

    double ra[4], rb[4];
    auto load = [&](int kt) {
        const double2 *ap = reinterpret_cast<const double2 *>(Ap + kt * BK);
        double2 x0 = ap[0], x1 = ap[1];
        ra[0] = x0.x; ra[1] = x0.y; ra[2] = x1.x; ra[3] = x1.y;
        const double *bp = Bp + (int64_t)kt * BK * ldb;
        if (b_full) {
            const double2 *bq = reinterpret_cast<const double2 *>(bp);
            double2 y0 = bq[0], y1 = bq[1];
            rb[0] = y0.x; rb[1] = y0.y; rb[2] = y1.x; rb[3] = y1.y;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) rb[c] = (n0 + b_n + c < N) ? bp[c] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < 4; ++c) As[buf][a_k + c][a_row] = ra[c];
#pragma unroll
        for (int c = 0; c < 4; ++c) Bs[buf][b_k][b_n + c] = rb[c];
    };

    dbl4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int KT = K / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < KT) load(kt + 1);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kk = ks * 4 + lane / 16;
            double af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[cur][kk][wm * (BM / WM) + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][kk][wn * (BN / WN) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
        }
        if (kt + 1 < KT) store(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * (BN / WN) + j * 16 + (lane & 15);
        const bool ok = col < N;
        int E = 0, par = 0;
        double w = 0.0;
        if (LORENTZ) {
            const int cc = ok ? col : 0;
            E = cc / la.ncp;
            const int jj = cc - E * la.ncp;
            par = jj & 1;
            w = la.omega[jj >> 1];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int row0 = m0 + wm * (BM / WM) + i * 16 + (lane >> 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 4 * r;
                double v = acc[i][j][r];
                if (LORENTZ) {
                    // L = n [1/(w - D + i eps) - 1/(w + D + i eps)], applied to
                    // the complex number held by this lane and its xor-1 partner.
                    const double other = __shfl_xor(v, 1);
                    const double D = la.Dlt[(int64_t)E * la.nv_pad + row];
                    const double d1 = w - D, d2 = w + D, e = la.eps;
                    const double s1 = 1.0 / (d1 * d1 + e * e), s2 = 1.0 / (d2 * d2 + e * e);
                    const double Lr = la.occ * (d1 * s1 - d2 * s2);
                    const double Li = la.occ * (-e * s1 + e * s2);
                    const double re = par ? other : v, im = par ? v : other;
                    v = par ? (re * Li + im * Lr) : (re * Lr - im * Li);
                }
                if (ok) C[(int64_t)row * ldc + col] = v;
            }
        }
    }
}

void launch_dgemm(Tracer *t, hipStream_t s, const char *name, int M, int N, int K,
                  const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                  double flops, double bytes) {
    const int tiles = (M / 64) * ((N + 63) / 64);
    LorentzArgs la{};
    const int m_fastest = (M / 64) <= ((N + 63) / 64);
    trace_begin(t, name, s);
    hipLaunchKernelGGL((k_dgemm<64, 64, 2, 2, false>), dim3(tiles), dim3(256), 0, s,
                       M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
    trace_end(t, s, flops, bytes);
}

void launch_dgemm_lorentz(Tracer *t, hipStream_t s, int M, int N, int K,
                          const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                          const double *Dlt, int nv_pad, const double *omega, double eps,
                          double occ, int ncp, double flops, double bytes) {
    const int tiles = (M / 64) * ((N + 63) / 64);
    LorentzArgs la{Dlt, omega, nv_pad, ncp, eps, occ};
    trace_begin(t, "virt_transform_lorentz", s);
    hipLaunchKernelGGL((k_dgemm<64, 64, 2, 2, true>), dim3(tiles), dim3(256), 0, s,
                       M, N, K, A, lda, B, ldb, C, ldc, 1, la);
    trace_end(t, s, flops, bytes);
}

// ------------------------------------------------------- (b1) occupied transform
// Tt[b][E*nc + j] = sum_{A in nbr(B)} sum_{a in A} Xo[a][E] dV[(k(A,B), a, b)][j]
// One workgroup: column atom B, 64 occupied states, 16 columns.  Wave w owns
// states 16w..16w+15 and every orbital b of B (one accumulator per b).
__global__ __launch_bounds__(256)
void k_occ_transform(BlockMapDev bm, const double *__restrict__ Xo, int no_pad,
                     const double *__restrict__ dV, double *__restrict__ Tt, int nc) {
    const int B = blockIdx.x, e0 = blockIdx.y * 64, j0 = blockIdx.z * JT;
    const int g0 = bm.col_gstart[B], g1 = bm.col_gstart[B + 1];
    const int boff = bm.atom_off[B], nB = bm.atom_off[B + 1] - boff;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    __shared__ double Xs[16][64 + 1];
    __shared__ double Ds[16][NB_MAX][JT];

    dbl4 acc[NB_MAX];
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int gc = g0; gc < g1; gc += 16) {
        {   // Xs: 16 gathered rows x 64 states, 4 per thread
            const int r = t / 16, c = (t % 16) * 4, g = gc + r;
            if (g < g1) {
                const double *src = Xo + (int64_t)bm.g_xrow[g] * no_pad + e0 + c;
                const double2 *p = reinterpret_cast<const double2 *>(src);
                double2 x0 = p[0], x1 = p[1];
                Xs[r][c] = x0.x; Xs[r][c + 1] = x0.y; Xs[r][c + 2] = x1.x; Xs[r][c + 3] = x1.y;
            } else {
                Xs[r][c] = 0.0; Xs[r][c + 1] = 0.0; Xs[r][c + 2] = 0.0; Xs[r][c + 3] = 0.0;
            }
        }
        for (int idx = t; idx < 16 * nB * JT; idx += 256) {
            const int r = idx / (nB * JT), rem = idx % (nB * JT);
            const int b = rem / JT, jj = rem % JT, g = gc + r, j = j0 + jj;
            double v = 0.0;
            if (g < g1 && j < nc) v = dV[(bm.g_ent[g] + b) * (int64_t)nc + j];
            Ds[r][b][jj] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const double a = Xs[kk][wv * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < NB_MAX; ++b)
                if (b < nB) acc[b] = mfma16(a, Ds[kk][b][lane & 15], acc[b]);
        }
        __syncthreads();
    }
    const int64_t ldT = (int64_t)no_pad * nc;
    const int j = j0 + (lane & 15);
    if (j < nc) {
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b) {
            if (b < nB) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int E = e0 + wv * 16 + 4 * r + (lane >> 4);
                    Tt[(int64_t)(boff + b) * ldT + (int64_t)E * nc + j] = acc[b][r];
                }
            }
        }
    }
}

void launch_occ_transform(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms,
                          const double *Xo, int no_pad, const double *dV, double *Tt,
                          int nc, const WorkSizes &ws) {
    dim3 grid(n_atoms, no_pad / 64, (nc + JT - 1) / JT);
    trace_begin(t, "occ_transform", s);
    hipLaunchKernelGGL(k_occ_transform, grid, dim3(256), 0, s, bm, Xo, no_pad, dV, Tt, nc);
    trace_end(t, s, 2.0 * ws.No * ws.nnzB * nc,
              8.0 * (ws.nnzB * nc + ws.N * ws.No + ws.N * ws.No * nc));
}

// ------------------------------------------------------ (b4) back to the pattern
// W[(k(A,B), a, b)][j] = sum_E Xo[a][E] Ut[b][E*nc + j] for (A, B) in the pattern.
// One workgroup: column atom B, 64 of its gathered rows (A, a), 16 columns.
__global__ __launch_bounds__(256)
void k_occ_back(BlockMapDev bm, const double *__restrict__ Xo, int no_pad,
                const double *__restrict__ Ut, double *__restrict__ W, int nc) {
    const int B = blockIdx.x, j0 = blockIdx.z * JT;
    const int g1 = bm.col_gstart[B + 1];
    const int g0 = bm.col_gstart[B] + blockIdx.y * 64;
    if (g0 >= g1) return;
    const int boff = bm.atom_off[B], nB = bm.atom_off[B + 1] - boff;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t ldT = (int64_t)no_pad * nc;
    __shared__ double Xs[64][16 + 1];
    __shared__ double Us[NB_MAX][16][JT];

    dbl4 acc[NB_MAX];
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int xr = t / 4, xc = (t % 4) * 4, xg = g0 + xr;
    const double *xsrc = (xg < g1) ? Xo + (int64_t)bm.g_xrow[xg] * no_pad + xc : nullptr;
    for (int E0 = 0; E0 < no_pad; E0 += 16) {
        if (xsrc) {
            const double2 *p = reinterpret_cast<const double2 *>(xsrc + E0);
            double2 x0 = p[0], x1 = p[1];
            Xs[xr][xc] = x0.x; Xs[xr][xc + 1] = x0.y; Xs[xr][xc + 2] = x1.x; Xs[xr][xc + 3] = x1.y;
        } else {
            Xs[xr][xc] = 0.0; Xs[xr][xc + 1] = 0.0; Xs[xr][xc + 2] = 0.0; Xs[xr][xc + 3] = 0.0;
        }
        for (int idx = t; idx < nB * 16 * JT; idx += 256) {
            const int b = idx / (16 * JT), rem = idx % (16 * JT);
            const int e = rem / JT, jj = rem % JT, j = j0 + jj;
            Us[b][e][jj] = (j < nc) ? Ut[(int64_t)(boff + b) * ldT + (int64_t)(E0 + e) * nc + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const double a = Xs[wv * 16 + (lane & 15)][kk];
#pragma unroll
            for (int b = 0; b < NB_MAX; ++b)
                if (b < nB) acc[b] = mfma16(a, Us[b][kk][lane & 15], acc[b]);
        }
        __syncthreads();
    }
    const int j = j0 + (lane & 15);
    if (j < nc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int g = g0 + wv * 16 + 4 * r + (lane >> 4);
            if (g < g1) {
                const int64_t base = bm.g_ent[g];
#pragma unroll
                for (int b = 0; b < NB_MAX; ++b)
                    if (b < nB) W[(base + b) * nc + j] = acc[b][r];
            }
        }
    }
}

void launch_occ_back(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms, int max_rows,
                     const double *Xo, int no_pad, const double *Ut, double *W, int nc,
                     const WorkSizes &ws) {
    dim3 grid(n_atoms, (max_rows + 63) / 64, (nc + JT - 1) / JT);
    trace_begin(t, "occ_back", s);
    hipLaunchKernelGGL(k_occ_back, grid, dim3(256), 0, s, bm, Xo, no_pad, Ut, W, nc);
    trace_end(t, s, 2.0 * ws.No * ws.nnzB * nc,
              8.0 * (ws.N * ws.No * nc + ws.N * ws.No + ws.nnzB * nc));
}

// ---------------------------------------------------------- (e) skinny K z
// Zout[mu][j] = sum_nu K[mu][nu] Zin[nu][j] for j < nc <= NC.  K streams from
// HBM once; each workgroup owns 16 rows (4 per wave) and stages 256-row
// chunks of Zin in LDS so Zin is read once per workgroup.
template <int NC>
__global__ __launch_bounds__(256)
void k_kmatvec_skinny(int P_pad, const double *__restrict__ K, const double *__restrict__ Zin,
                      double *__restrict__ Zout, int nc) {
    __shared__ double Zs[256][NC];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row0 = blockIdx.x * 16 + wv * 4;
    double acc[4][NC];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[r][j] = 0.0;
    for (int nu0 = 0; nu0 < P_pad; nu0 += 256) {
        for (int idx = t; idx < 256 * NC; idx += 256) {
            const int r = idx / NC, j = idx % NC, nu = nu0 + r;
            Zs[r][j] = (nu < P_pad && j < nc) ? Zin[(int64_t)nu * nc + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int nl = c * 64 + lane, nu = nu0 + nl;
            if (nu < P_pad) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double kv = K[(int64_t)(row0 + r) * P_pad + nu];
#pragma unroll
                    for (int j = 0; j < NC; ++j) acc[r][j] += kv * Zs[nl][j];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            double v = acc[r][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && j < nc) Zout[(int64_t)(row0 + r) * nc + j] = v;
        }
}

void launch_kmatvec_skinny(Tracer *t, hipStream_t s, int P_pad, const double *K,
                           const double *Zin, double *Zout, int nc, double P) {
    dim3 grid(P_pad / 16);
    trace_begin(t, "kernel_matvec", s);
    if (nc <= 2)
        hipLaunchKernelGGL(k_kmatvec_skinny<2>, grid, dim3(256), 0, s, P_pad, K, Zin, Zout, nc);
    else if (nc <= 4)
        hipLaunchKernelGGL(k_kmatvec_skinny<4>, grid, dim3(256), 0, s, P_pad, K, Zin, Zout, nc);
    else if (nc <= 8)
        hipLaunchKernelGGL(k_kmatvec_skinny<8>, grid, dim3(256), 0, s, P_pad, K, Zin, Zout, nc);
    else
        hipLaunchKernelGGL(k_kmatvec_skinny<16>, grid, dim3(256), 0, s, P_pad, K, Zin, Zout, nc);
    trace_end(t, s, 2.0 * P * P * nc, 8.0 * (P * P + 2.0 * P * nc));
}

}  // namespace chi0
