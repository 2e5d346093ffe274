// Matrix-core kernels of the orbital transforms (Sec. 4.2, Table t:flops steps
// 2-5) and the kernel matrix-vector product (Sec. 4.1), for FP64 and FP32.
//
// A 16 x 16 output tile per K step of 4 on 64-lane wavefronts, lane l = 0..63:
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): element r of lane l holds D[row(l, r)][l % 16]
// FP64 uses v_mfma_f64_4x4x4_4b_f64: four 4x4x4 products per instruction,
// lane l = 16 h + 4 q + p holding A[q-th block][p][h], B[block q][h][p] and
// D[block q][h][p].  Issuing one instruction per 4-row strip r of the tile,
// with block q = the 4-column group of B, makes B and D the same lanes as a
// 16x16x4 product:  A fragment r holds A[4r + l % 4][l / 16], and
// row(l, r) = 4r + l/16.  On gfx950 this form runs at ~72 TFLOP/s against
// ~50 for v_mfma_f64_16x16x4f64 (register-only throughput probes).
// FP32 uses v_mfma_f32_16x16x4f32: A[l % 16][l / 16], row(l, r) = 4(l/16) + r.
// (Lane layouts checked on gfx950 with one-hot lane probes.)
#include "common.h"

#include <algorithm>
#include <cmath>

namespace chi0 {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// NA A fragments per 16 x 16 tile and K step; a_row(l, r) is the tile row
// that lane l supplies in fragment r.
template <class T> struct Mma;
template <> struct Mma<double> {
    typedef dbl4 acc;
    static constexpr int NA = 4;
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ int a_row(int lane, int r) { return 4 * r + (lane & 3); }
    static __device__ __forceinline__ acc op(const double (&a)[NA], double b, acc c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[r], b, c[r], 0, 0, 0);
        return c;
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
// The gathered occupied transforms keep the single 16x16x4 FP64 product per
// tile (A[l % 16][l / 16]): with a dozen accumulators per wave they are not
// bound by the MFMA issue rate, and the four A fragments of the 4-block form
// made them slower.
struct Mma16d {
    typedef dbl4 acc;
    static constexpr int NA = 1;
    static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ int a_row(int lane, int) { return lane & 15; }
    static __device__ __forceinline__ acc op(const double (&a)[NA], double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mma<float> {
    typedef flt4 acc;
    static constexpr int NA = 1;
    static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ int a_row(int lane, int) { return lane & 15; }
    static __device__ __forceinline__ acc op(const float (&a)[NA], float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// four consecutive elements (16 B aligned for float, 2 x 16 B for double)
__device__ __forceinline__ void load4(const double *p, double *v) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float *p, float *v) {
    const float4 a = reinterpret_cast<const float4 *>(p)[0];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
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
// Split-K: blockIdx.y selects a K range of length K (the per-split length);
// A and B are advanced by it and each split writes raw partial sums to its
// own C slice (C + split * M * ldc), summed later by k_splitk_reduce.
// The tile shape (BM x BN, WM x WN wavefronts) changes only which workgroup
// computes an element, never the order of its k accumulation, so every tile
// variant gives bit-identical results and the autotuner may pick any of them.
template <class T, int BM, int BN, int WM, int WN, bool LORENTZ, int BK = 16>
__global__ __launch_bounds__(WM * WN * 64)
void k_dgemm(int M, int N, int K, const T *__restrict__ A, int lda,
             const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc,
             int m_fastest, LorentzArgs la) {
    A += (int64_t)blockIdx.y * K;
    B += (int64_t)blockIdx.y * K * ldb;
    C += (int64_t)blockIdx.y * M * ldc;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 16;
    constexpr int TN = BN / WN / 16;
    constexpr int CA = BM * (BK / 4) / NT;   // 4-element A chunks per thread per tile
    constexpr int CB = BK * (BN / 4) / NT;   // 4-element B chunks per thread per tile
    static_assert(CA >= 1 && CB >= 1 && CA * NT == BM * (BK / 4) && CB * NT == BK * (BN / 4),
                  "tile shape must split into whole 4-element chunks per thread");
    __shared__ T As[2][BK][BM + 1];
    __shared__ T Bs[2][BK][BN];

    const int ntm = M / BM, ntn = (N + BN - 1) / BN;
    const int tile = xcd_remap(blockIdx.x, ntm * ntn);
    const int tm = m_fastest ? tile % ntm : tile / ntn;
    const int tn = m_fastest ? tile / ntm : tile % ntn;
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % WM, wn = wv / WM;

    // global -> register mapping: chunk q of a thread is chunk t + q NT of the tile
    int a_row[CA], a_k[CA], b_k[CB], b_n[CB];
#pragma unroll
    for (int q = 0; q < CA; ++q) {
        const int ch = t + q * NT;
        a_row[q] = ch / (BK / 4);
        a_k[q] = (ch % (BK / 4)) * 4;
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
        const int ch = t + q * NT;
        b_k[q] = ch / (BN / 4);
        b_n[q] = (ch % (BN / 4)) * 4;
    }

    T ra[CA][4], rb[CB][4];
    auto load = [&](int kt) {
#pragma unroll
        for (int q = 0; q < CA; ++q) load4(A + (int64_t)(m0 + a_row[q]) * lda + kt * BK + a_k[q], ra[q]);
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            const T *bp = B + (int64_t)(kt * BK + b_k[q]) * ldb + n0 + b_n[q];
            if (n0 + b_n[q] + 3 < N) {
                load4(bp, rb[q]);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) rb[q][c] = (n0 + b_n[q] + c < N) ? bp[c] : T(0);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < CA; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) As[buf][a_k[q] + c][a_row[q]] = ra[q][c];
#pragma unroll
        for (int q = 0; q < CB; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) Bs[buf][b_k[q]][b_n[q] + c] = rb[q][c];
    };

    typename Mma<T>::acc acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::zero();

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
            T af[TM][Mma<T>::NA], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int r = 0; r < Mma<T>::NA; ++r)
                    af[i][r] = As[cur][kk][wm * (BM / WM) + i * 16 + Mma<T>::a_row(lane, r)];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][kk][wn * (BN / WN) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::op(af[i], bf[j], acc[i][j]);
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
            const int rbase = m0 + wm * (BM / WM) + i * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rbase + Mma<T>::row(lane, r);
                T v = acc[i][j][r];
                if (LORENTZ) {
                    // L = n [1/(w - D + i eps) - 1/(w + D + i eps)] (in FP64), applied
                    // to the complex number held by this lane and its xor-1 partner;
                    // the pair shares the two reciprocals (one computed by each lane).
                    const T other = __shfl_xor(v, 1);
                    const double D = la.Dlt[(int64_t)E * la.nv_pad + row];
                    const double d1 = w - D, d2 = w + D, e = la.eps;
                    const double dm = par ? d2 : d1;
                    const double sm = 1.0 / (dm * dm + e * e), so = __shfl_xor(sm, 1);
                    const double s1 = par ? so : sm, s2 = par ? sm : so;
                    const double Lr = la.occ * (d1 * s1 - d2 * s2);
                    const double Li = la.occ * (-e * s1 + e * s2);
                    const double re = par ? (double)other : (double)v, im = par ? (double)v : (double)other;
                    v = (T)(par ? (re * Li + im * Lr) : (re * Lr - im * Li));
                }
                // the output is read by the next kernel only: a streaming store
                if (ok) __builtin_nontemporal_store(v, &C[(int64_t)row * ldc + col]);
            }
        }
    }
}

// C = sum over splits of the partial products; optional Lorentzian epilogue.
template <class T>
__global__ __launch_bounds__(256)
void k_splitk_reduce(int M, int N, int S, const T *__restrict__ part, int64_t slice,
                     T *__restrict__ C, int ldc, int lorentz, LorentzArgs la) {
    const int64_t npair = (int64_t)M * ((N + 1) / 2);
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < npair;
         idx += (int64_t)gridDim.x * 256) {
        const int row = (int)(idx / ((N + 1) / 2));
        const int col = 2 * (int)(idx % ((N + 1) / 2));
        const int64_t o = (int64_t)row * ldc + col;
        const int64_t op = (int64_t)row * N + col;
        const bool two = col + 1 < N;
        double re = 0.0, im = 0.0;
        for (int s2 = 0; s2 < S; ++s2) {
            re += (double)part[s2 * slice + op];
            if (two) im += (double)part[s2 * slice + op + 1];
        }
        if (lorentz) {
            const int E = col / la.ncp, jj = col - E * la.ncp;
            const double w = la.omega[jj >> 1];
            const double D = la.Dlt[(int64_t)E * la.nv_pad + row];
            const double d1 = w - D, d2 = w + D, e = la.eps;
            const double s1 = 1.0 / (d1 * d1 + e * e), s2 = 1.0 / (d2 * d2 + e * e);
            const double Lr = la.occ * (d1 * s1 - d2 * s2), Li = la.occ * (-e * s1 + e * s2);
            const double r2 = re * Lr - im * Li, i2 = re * Li + im * Lr;
            re = r2;
            im = i2;
        }
        C[o] = (T)re;
        if (two) C[o + 1] = (T)im;
    }
}

// Number of K splits: enough workgroups to fill 256 CUs a few times over,
// each split keeping >= 4 K tiles of 16; limited by the scratch capacity.  The
// splits have equal lengths *ks of whole tiles; S *ks may exceed K (the last
// split then sums zero padding) but not kpad, the operands' K extent.
static int choose_splits(int M, int N, int K, int kpad, size_t scratch_elems, int *ks) {
    const int tiles = (M / 64) * ((N + 63) / 64);
    const int KT = K / 16;
    int S = 1;
    while (S < 16 && tiles * S < 1024) {
        const int S2 = 2 * S, kt2 = (KT + S2 - 1) / S2;
        if (kt2 < 4 || (int64_t)S2 * kt2 * 16 > kpad || (size_t)S2 * M * (size_t)N > scratch_elems) break;
        S = S2;
    }
    *ks = (KT + S - 1) / S * 16;
    return S;
}

template <class T>
static void reduce_splits(Tracer *t, hipStream_t s, int M, int N, int S, const T *scratch, T *C,
                          int ldc, bool lorentz, const LorentzArgs &la) {
    const int64_t npair = (int64_t)M * ((N + 1) / 2);
    int64_t blocks = (npair + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    trace_begin(t, "splitk_reduce", s);
    hipLaunchKernelGGL(k_splitk_reduce<T>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, S, scratch,
                       (int64_t)M * N, C, ldc, lorentz ? 1 : 0, la);
    trace_end(t, s, (double)S * M * N, (double)sizeof(T) * ((double)S + 1.0) * M * N);
}

const char *const kGemmVariantNames[GEMM_VARIANTS] = {"64x64", "64x128", "128x64", "128x128",
                                                      "64x64/k32", "64x128/k32"};
static const int kVarBM[GEMM_VARIANTS] = {64, 64, 128, 128, 64, 64};
static const int kVarBK[GEMM_VARIANTS] = {16, 16, 16, 16, 32, 32};

GemmTuner::~GemmTuner() {
    for (hipEvent_t &e : ev)
        if (e) (void)hipEventDestroy(e);
}

template <class T, bool LZ>
static void launch_variant(int v, hipStream_t s, dim3 grid_s, int M, int N, int K, const T *A, int lda,
                           const T *B, int ldb, T *C, int ldc, int m_fastest, const LorentzArgs &la) {
    const int S = grid_s.y;
    auto tiles = [&](int bm, int bn) { return (unsigned)((M / bm) * ((N + bn - 1) / bn)); };
    switch (v) {
    case 1:
        hipLaunchKernelGGL((k_dgemm<T, 64, 128, 2, 2, LZ>), dim3(tiles(64, 128), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    case 2:
        hipLaunchKernelGGL((k_dgemm<T, 128, 64, 2, 2, LZ>), dim3(tiles(128, 64), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    case 3:
        hipLaunchKernelGGL((k_dgemm<T, 128, 128, 2, 2, LZ>), dim3(tiles(128, 128), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    case 4:
        hipLaunchKernelGGL((k_dgemm<T, 64, 64, 2, 2, LZ, 32>), dim3(tiles(64, 64), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    case 5:
        hipLaunchKernelGGL((k_dgemm<T, 64, 128, 2, 2, LZ, 32>), dim3(tiles(64, 128), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    default:
        hipLaunchKernelGGL((k_dgemm<T, 64, 64, 2, 2, LZ>), dim3(tiles(64, 64), S), dim3(256), 0, s,
                           M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        break;
    }
}

// Variant for this call: the tuned one for its key, tuning first if the key is new.
template <class T, bool LZ>
static int pick_variant(GemmTuner *tu, hipStream_t s, const char *name, int S, int M, int N, int K,
                        const T *A, int lda, const T *B, int ldb, T *C, int ldc, int m_fastest,
                        const LorentzArgs &la) {
    if (!tu) return 0;
    if (tu->force >= 0 && tu->force < GEMM_VARIANTS)
        return (M % kVarBM[tu->force] == 0 && K % kVarBK[tu->force] == 0) ? tu->force : 0;
    if (!tu->enabled) return 0;
    const int nb = (int)std::floor(2.0 * std::log2((double)std::max(N, 1)));
    const std::string key = std::string(name) + (sizeof(T) == 8 ? "" : "_f32") + " M=" + std::to_string(M) +
                            " K=" + std::to_string(K * S) + " S=" + std::to_string(S) + " N~2^" +
                            std::to_string(nb / 2) + (nb % 2 ? ".5" : "");
    auto it = tu->table.find(key);
    if (it != tu->table.end()) return it->second.variant;
    GemmTuner::Entry e;
    for (hipEvent_t &ev : tu->ev)
        if (!ev && hipEventCreate(&ev) != hipSuccess) return 0;
    float best = 0.f;
    for (int v = 0; v < GEMM_VARIANTS; ++v) {
        if (M % kVarBM[v] != 0 || K % kVarBK[v] != 0) continue;
        launch_variant<T, LZ>(v, s, dim3(1, S), M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        // best of three timed launches: one launch's time varies by several per cent
        float tmin = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(tu->ev[0], s);
            launch_variant<T, LZ>(v, s, dim3(1, S), M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
            (void)hipEventRecord(tu->ev[1], s);
            float ms = 0.f;
            if (hipEventSynchronize(tu->ev[1]) != hipSuccess ||
                hipEventElapsedTime(&ms, tu->ev[0], tu->ev[1]) != hipSuccess)
                return 0;
            tmin = rep == 0 ? ms : std::min(tmin, ms);
        }
        e.us[v] = 1e3f * tmin;
        if (best == 0.f || e.us[v] < best) {
            best = e.us[v];
            e.variant = v;
        }
    }
    tu->table.emplace(key, e);
    return e.variant;
}

template <class T>
static void gemm_any(Tracer *t, hipStream_t s, const char *name, int M, int N, int K, int kpad,
                     const T *A, int lda, const T *B, int ldb, T *C, int ldc,
                     double flops, double bytes, bool lorentz, const LorentzArgs &la,
                     void *scratch, size_t scratch_bytes, GemmTuner *tu) {
    int ks = K;
    const int S = scratch ? choose_splits(M, N, K, kpad, scratch_bytes / sizeof(T), &ks) : 1;
    const int m_fastest = (M / 64) <= ((N + 63) / 64);
    if (S == 1) {
        if (lorentz) {
            const int v = pick_variant<T, true>(tu, s, name, 1, M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
            trace_begin(t, name, s);
            launch_variant<T, true>(v, s, dim3(1, 1), M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        } else {
            const int v = pick_variant<T, false>(tu, s, name, 1, M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
            trace_begin(t, name, s);
            launch_variant<T, false>(v, s, dim3(1, 1), M, N, K, A, lda, B, ldb, C, ldc, m_fastest, la);
        }
        trace_end(t, s, flops, bytes);
        return;
    }
    // partial products with ldc = N into scratch, then the reduction (+ epilogue)
    T *part = static_cast<T *>(scratch);
    const int v = pick_variant<T, false>(tu, s, name, S, M, N, ks, A, lda, B, ldb, part, N, m_fastest, la);
    trace_begin(t, name, s);
    launch_variant<T, false>(v, s, dim3(1, S), M, N, ks, A, lda, B, ldb, part, N, m_fastest, la);
    trace_end(t, s, flops, bytes);
    reduce_splits<T>(t, s, M, N, S, part, C, ldc, lorentz, la);
}

void launch_dgemm(Tracer *t, hipStream_t s, const char *name, int M, int N, int K, int kpad,
                  const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                  double flops, double bytes, double *scratch, size_t scratch_doubles, GemmTuner *tu) {
    LorentzArgs la{};
    gemm_any<double>(t, s, name, M, N, K, kpad, A, lda, B, ldb, C, ldc, flops, bytes, false, la, scratch,
                     scratch_doubles * sizeof(double), tu);
}

void launch_dgemm_lorentz(Tracer *t, hipStream_t s, int M, int N, int K, int kpad,
                          const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                          const double *Dlt, int nv_pad, const double *omega, double eps,
                          double occ, int ncp, double flops, double bytes, double *scratch,
                          size_t scratch_doubles, GemmTuner *tu) {
    LorentzArgs la{Dlt, omega, nv_pad, ncp, eps, occ};
    gemm_any<double>(t, s, "virt_transform_lorentz", M, N, K, kpad, A, lda, B, ldb, C, ldc, flops, bytes,
                     true, la, scratch, scratch_doubles * sizeof(double), tu);
}

void launch_splitk_reduce_f32(Tracer *t, hipStream_t s, int M, int N, int S, const float *part,
                              float *C, int ldc, const LorentzArgs *la) {
    LorentzArgs none{};
    reduce_splits<float>(t, s, M, N, S, part, C, ldc, la != nullptr, la ? *la : none);
}

void launch_sgemm(Tracer *t, hipStream_t s, const char *name, int M, int N, int K,
                  const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                  double flops, double bytes, const LorentzArgs *la, void *scratch,
                  size_t scratch_bytes, GemmTuner *tu) {
    LorentzArgs none{};
    gemm_any<float>(t, s, name, M, N, K, K, A, lda, B, ldb, C, ldc, flops, bytes, la != nullptr,
                    la ? *la : none, scratch, scratch_bytes, tu);
}

template <class T> struct OccMma { typedef Mma<T> type; };
template <> struct OccMma<double> { typedef Mma16d type; };

// ------------------------------------------------------- (b1) occupied transform
// The gathered transforms multiply by one atom's orbitals b at a time, for every
// column j; their output columns are the packed pairs n = b nc + j of the column
// atom (nB nc of them), cut into 16-column MFMA tiles, OCC_NT tiles per
// workgroup.  A few right-hand sides therefore fill the tiles: one complex
// vector (nc = 2) on a 9-orbital atom is 18 pairs, two tiles, not nine tiles of
// which 2 columns are used.
constexpr int OCC_NT = 9;              // 16-column tiles per workgroup
constexpr int OCC_NW = 16 * OCC_NT;    // packed (b, j) pairs per workgroup

// Tt[b][E*nc + j] = sum_{A in nbr(B)} sum_{a in A} Xo[a][E] dV[(k(A,B), a, b)][j]
// One workgroup: column atom B, 64 occupied states, OCC_NW packed pairs.  Wave w
// owns states 16w..16w+15.  The gathered rows come in chunks of 16; the next
// chunk's global loads are issued before the current chunk's MFMAs so their
// latency overlaps the arithmetic.  Row g of dV holds the pairs of B
// contiguously (dV[(k, a, b)][j] = dV[k_a nc + n]), so a chunk's pairs are one
// coalesced run per gathered row.  T is the arithmetic type (FP64, or FP32 for
// the low-precision operator); dV is always FP64 and is rounded to T when staged.
template <class T>
__global__ __launch_bounds__(256)
void k_occ_transform(BlockMapDev bm, const T *__restrict__ Xo, int no_pad,
                     const double *__restrict__ dV, T *__restrict__ Tt, int nc) {
    typedef typename OccMma<T>::type MM;
    const int B = blockIdx.x, e0 = blockIdx.y * 64, n0 = blockIdx.z * OCC_NW;
    const int g0 = bm.col_gstart[B], g1 = bm.col_gstart[B + 1];
    const int boff = bm.atom_off[B], nB = bm.atom_off[B + 1] - boff;
    const int nn = nB * nc;
    if (n0 >= nn) return;
    const int ntile = min(OCC_NT, (nn - n0 + 15) / 16);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    __shared__ T Xs[16][64 + 1];
    __shared__ T Ds[16][OCC_NW];

    typename MM::acc acc[OCC_NT];
#pragma unroll
    for (int i = 0; i < OCC_NT; ++i) acc[i] = MM::zero();

    // register staging of one chunk: 4 X values and OCC_NT dV values of one row
    const int xr = t / 16, xc = (t % 16) * 4;
    const int dr = t / 16, dn = t % 16;
    T xv[4], dv[OCC_NT];
    auto fetch = [&](int gc) {
        const int gx = gc + xr;
        xv[0] = xv[1] = xv[2] = xv[3] = T(0);
        if (gx < g1) load4(Xo + (int64_t)bm.g_xrow[gx] * no_pad + e0 + xc, xv);
        const int gd = gc + dr;
        const double *src = dV + (gd < g1 ? (int64_t)bm.g_ent[gd] * nc : 0) + n0 + dn;
#pragma unroll
        for (int i = 0; i < OCC_NT; ++i)
            dv[i] = (gd < g1 && n0 + 16 * i + dn < nn) ? (T)src[16 * i] : T(0);
    };
    fetch(g0);
    for (int gc = g0; gc < g1; gc += 16) {
        Xs[xr][xc] = xv[0]; Xs[xr][xc + 1] = xv[1]; Xs[xr][xc + 2] = xv[2]; Xs[xr][xc + 3] = xv[3];
#pragma unroll
        for (int i = 0; i < OCC_NT; ++i) Ds[dr][16 * i + dn] = dv[i];
        __syncthreads();
        if (gc + 16 < g1) fetch(gc + 16);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            T a[MM::NA];
#pragma unroll
            for (int r = 0; r < MM::NA; ++r) a[r] = Xs[kk][wv * 16 + MM::a_row(lane, r)];
#pragma unroll
            for (int i = 0; i < OCC_NT; ++i)
                if (i < ntile) acc[i] = MM::op(a, Ds[kk][16 * i + (lane & 15)], acc[i]);
        }
        __syncthreads();
    }
    const int64_t ldT = (int64_t)no_pad * nc;
#pragma unroll
    for (int i = 0; i < OCC_NT; ++i) {
        const int n = n0 + 16 * i + (lane & 15);
        if (i < ntile && n < nn) {
            const int b = n / nc, j = n - b * nc;
            T *dst = Tt + (int64_t)(boff + b) * ldT + j;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int E = e0 + wv * 16 + MM::row(lane, r);
                dst[(int64_t)E * nc] = acc[i][r];
            }
        }
    }
}

static inline int occ_pair_blocks(const BlockMapDev &bm, int nc) {
    return (bm.nb_max * nc + OCC_NW - 1) / OCC_NW;
}

template <class T>
static void occ_transform_any(Tracer *t, hipStream_t s, const char *name, const BlockMapDev &bm,
                              int n_atoms, const T *Xo, int no_pad, const double *dV, T *Tt, int nc,
                              const WorkSizes &ws) {
    dim3 grid(n_atoms, no_pad / 64, occ_pair_blocks(bm, nc));
    trace_begin(t, name, s);
    hipLaunchKernelGGL((k_occ_transform<T>), grid, dim3(256), 0, s, bm, Xo, no_pad, dV, Tt, nc);
    trace_end(t, s, 2.0 * ws.No * ws.nnzB * nc,
              8.0 * ws.nnzB * nc + sizeof(T) * (ws.N * ws.No + ws.N * ws.No * nc));
}

void launch_occ_transform(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms,
                          const double *Xo, int no_pad, const double *dV, double *Tt,
                          int nc, const WorkSizes &ws) {
    occ_transform_any<double>(t, s, "occ_transform", bm, n_atoms, Xo, no_pad, dV, Tt, nc, ws);
}

void launch_occ_transform_f32(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms,
                              const float *Xo, int no_pad, const double *dV, float *Tt,
                              int nc, const WorkSizes &ws) {
    occ_transform_any<float>(t, s, "occ_transform_f32", bm, n_atoms, Xo, no_pad, dV, Tt, nc, ws);
}

// ------------------------------------------------------ (b4) back to the pattern
// W[(k(A,B), a, b)][j] = sum_E Xo[a][E] Ut[b][E*nc + j] for (A, B) in the pattern.
// One workgroup: column atom B, 64 of its gathered rows (A, a), OCC_NW packed
// pairs n = b nc + j; the occupied states E < no_sum come in chunks of 16 with the next
// chunk's global loads issued before the current chunk's MFMAs.  A wave whose
// 16 rows lie past the atom's last gathered row stages its share of the
// operands and skips the MFMAs.  Accumulation in T; W is FP64.
template <class T>
__global__ __launch_bounds__(256)
void k_occ_back(BlockMapDev bm, const T *__restrict__ Xo, int no_pad, int no_sum,
                const T *__restrict__ Ut, double *__restrict__ W, int nc) {
    typedef typename OccMma<T>::type MM;
    const int B = blockIdx.x, n0 = blockIdx.z * OCC_NW;
    const int g1 = bm.col_gstart[B + 1];
    const int g0 = bm.col_gstart[B] + blockIdx.y * 64;
    if (g0 >= g1) return;
    const int boff = bm.atom_off[B], nB = bm.atom_off[B + 1] - boff;
    const int nn = nB * nc;
    if (n0 >= nn) return;
    const int ntile = min(OCC_NT, (nn - n0 + 15) / 16);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const bool live = g0 + wv * 16 < g1;
    const int64_t ldT = (int64_t)no_pad * nc;
    __shared__ T Xs[64][16 + 1];
    __shared__ T Us[16][OCC_NW];

    typename MM::acc acc[OCC_NT];
#pragma unroll
    for (int i = 0; i < OCC_NT; ++i) acc[i] = MM::zero();

    const int xr = t / 4, xc = (t % 4) * 4, xg = g0 + xr;
    const T *xsrc = (xg < g1) ? Xo + (int64_t)bm.g_xrow[xg] * no_pad + xc : nullptr;
    // pair i of this thread: n = n0 + 16 i + un, at Ut[(boff + b) ldT + E nc + j]
    const int ue = t / 16, un = t % 16;
    int64_t uoff[OCC_NT];
#pragma unroll
    for (int i = 0; i < OCC_NT; ++i) {
        const int n = n0 + 16 * i + un;
        const int b = n / nc, j = n - b * nc;
        uoff[i] = n < nn ? (int64_t)(boff + b) * ldT + (int64_t)ue * nc + j : -1;
    }
    T xv[4], uv[OCC_NT];
    auto fetch = [&](int E0) {
        xv[0] = xv[1] = xv[2] = xv[3] = T(0);
        if (xsrc) load4(xsrc + E0, xv);
#pragma unroll
        for (int i = 0; i < OCC_NT; ++i)
            uv[i] = uoff[i] >= 0 ? Ut[uoff[i] + (int64_t)E0 * nc] : T(0);
    };
    fetch(0);
    for (int E0 = 0; E0 < no_sum; E0 += 16) {
        Xs[xr][xc] = xv[0]; Xs[xr][xc + 1] = xv[1]; Xs[xr][xc + 2] = xv[2]; Xs[xr][xc + 3] = xv[3];
#pragma unroll
        for (int i = 0; i < OCC_NT; ++i) Us[ue][16 * i + un] = uv[i];
        __syncthreads();
        if (E0 + 16 < no_sum) fetch(E0 + 16);
        if (live) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = ks * 4 + (lane >> 4);
                T a[MM::NA];
#pragma unroll
                for (int r = 0; r < MM::NA; ++r) a[r] = Xs[wv * 16 + MM::a_row(lane, r)][kk];
#pragma unroll
                for (int i = 0; i < OCC_NT; ++i)
                    if (i < ntile) acc[i] = MM::op(a, Us[kk][16 * i + (lane & 15)], acc[i]);
            }
        }
        __syncthreads();
    }
    if (!live) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int g = g0 + wv * 16 + MM::row(lane, r);
        if (g < g1) {
            double *dst = W + (int64_t)bm.g_ent[g] * nc;   // row (k, a, b) = g_ent[g] + b: column b nc + j
#pragma unroll
            for (int i = 0; i < OCC_NT; ++i) {
                const int n = n0 + 16 * i + (lane & 15);
                if (i < ntile && n < nn) dst[n] = (double)acc[i][r];
            }
        }
    }
}

template <class T>
static void occ_back_any(Tracer *t, hipStream_t s, const char *name, const BlockMapDev &bm,
                         int n_atoms, int max_rows, const T *Xo, int no_pad, int no_sum, const T *Ut,
                         double *W, int nc, const WorkSizes &ws) {
    dim3 grid(n_atoms, (max_rows + 63) / 64, occ_pair_blocks(bm, nc));
    trace_begin(t, name, s);
    hipLaunchKernelGGL((k_occ_back<T>), grid, dim3(256), 0, s, bm, Xo, no_pad, no_sum, Ut, W, nc);
    trace_end(t, s, 2.0 * ws.No * ws.nnzB * nc,
              sizeof(T) * (ws.N * ws.No * nc + ws.N * ws.No) + 8.0 * ws.nnzB * nc);
}

void launch_occ_back(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms, int max_rows,
                     const double *Xo, int no_pad, int no_sum, const double *Ut, double *W, int nc,
                     const WorkSizes &ws) {
    occ_back_any<double>(t, s, "occ_back", bm, n_atoms, max_rows, Xo, no_pad, no_sum, Ut, W, nc, ws);
}

void launch_occ_back_f32(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms, int max_rows,
                         const float *Xo, int no_pad, int no_sum, const float *Ut, double *W, int nc,
                         const WorkSizes &ws) {
    occ_back_any<float>(t, s, "occ_back_f32", bm, n_atoms, max_rows, Xo, no_pad, no_sum, Ut, W, nc, ws);
}

// ---------------------------------------------------------- (e) skinny K z
// Zout[mu][j] = sum_nu K[mu][nu] Zin[nu][j] for a few columns j < nc: K
// streams from HBM once per product.
// Up to two right-hand sides (nc = 1..4 real columns): a wavefront owns RW
// rows and every lane reads 16-byte pairs of K columns, U pairs of chunks in
// flight per row; the two Zin rows a lane needs (2 nc doubles, contiguous) are
// read through the cache.  Four times the wavefronts of the LDS-staged form,
// with no barrier in the loop.
template <int NC, int RW>
__global__ __launch_bounds__(256)
void k_kmatvec_lanes(int P_pad, const double *__restrict__ K, const double *__restrict__ Zin,
                     double *__restrict__ Zout) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + wv) * RW;
    double acc[RW][NC];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[r][j] = 0.0;
    for (int c0 = 2 * lane; c0 < P_pad; c0 += 128 * U) {
        double2 kv[U][RW];
        double2 zv[U][NC];   // Zin rows nu and nu + 1: 2 NC doubles
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int nu = c0 + 128 * u;
            const bool ok = nu < P_pad;
#pragma unroll
            for (int r = 0; r < RW; ++r)
                kv[u][r] = ok ? *reinterpret_cast<const double2 *>(K + (int64_t)(row0 + r) * P_pad + nu)
                              : make_double2(0.0, 0.0);
#pragma unroll
            for (int h = 0; h < NC; ++h)
                zv[u][h] = ok ? reinterpret_cast<const double2 *>(Zin + (int64_t)nu * NC)[h]
                              : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double *z = reinterpret_cast<const double *>(zv[u]);   // z[0..NC): row nu, z[NC..2NC): nu + 1
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int j = 0; j < NC; ++j) acc[r][j] += kv[u][r].x * z[j] + kv[u][r].y * z[NC + j];
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            double v = acc[r][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) Zout[(int64_t)(row0 + r) * NC + j] = v;
        }
}

constexpr int KMV_RT = 2;   // 16-row tiles per workgroup of the MFMA form
constexpr int KMV_U = 8;    // column pairs per lane and row tile in flight

// 5..32 real columns on the FP64 matrix cores (CT 16-column tiles).  A
// workgroup owns 16 RT rows;
// its four waves split the reduction over nu in interleaved chunks of 8 U
// columns and add their 16x16 accumulators in a fixed order through LDS at
// the end.  Each lane streams K as 16-byte loads of two adjacent columns; the
// two columns feed two 16x16x4 MFMAs whose k slots are the lanes' even and odd
// columns, with Zin rows taken in the same order.  Zin (P_pad x nc, a few MB)
// is read through the cache; no barrier in the loop.  With PF the loads of the
// wave's next chunk are issued before the MFMAs of the current one (one
// 16-column tile: 4.3-4.4 TB/s against 4.0-4.2 without, on the 12.4k-product
// kernel, 1.2 GB; with two tiles the doubled registers make it slower).
// (LDS-staged form: 0.25-3.4 TB/s; non-temporal loads of K were 10 % slower.)
template <int RT, int CT, int U, bool PF>
__global__ __launch_bounds__(256)
void k_kmatvec_mfma(int P_pad, const double *__restrict__ K, const double *__restrict__ Zin,
                    double *__restrict__ Zout, int nc) {
    __shared__ dbl4 red[3][RT][CT][64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row0 = blockIdx.x * 16 * RT;
    const int lr = lane & 15, lk = lane >> 4;
    dbl4 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};
    constexpr int KW = 8 * U;
    double2 a[U][RT];
    double b0[U][CT], b1[U][CT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = k0 + 8 * u + 2 * lk;   // even; P_pad is a multiple of 64
            const bool ok = kk < P_pad;
#pragma unroll
            for (int r = 0; r < RT; ++r)
                a[u][r] = ok ? *reinterpret_cast<const double2 *>(K + (int64_t)(row0 + 16 * r + lr) * P_pad + kk)
                              : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int col = 16 * c + lr;
                b0[u][c] = (ok && col < nc) ? Zin[(int64_t)kk * nc + col] : 0.0;
                b1[u][c] = (ok && col < nc) ? Zin[(int64_t)(kk + 1) * nc + col] : 0.0;
            }
        }
    };
    auto mma = [&](const double2 (&ca)[U][RT], const double (&c0)[U][CT], const double (&c1)[U][CT]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][r].x, c0[u][c], acc[r][c], 0, 0, 0);
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][r].y, c1[u][c], acc[r][c], 0, 0, 0);
                }
    };
    if constexpr (PF) {
        int k0 = wv * KW;
        if (k0 < P_pad) fetch(k0);
        for (; k0 < P_pad; k0 += 4 * KW) {
            double2 ca[U][RT];
            double c0[U][CT], c1[U][CT];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int r = 0; r < RT; ++r) ca[u][r] = a[u][r];
#pragma unroll
                for (int c = 0; c < CT; ++c) { c0[u][c] = b0[u][c]; c1[u][c] = b1[u][c]; }
            }
            if (k0 + 4 * KW < P_pad) fetch(k0 + 4 * KW);
            mma(ca, c0, c1);
        }
    } else {
        for (int k0 = wv * KW; k0 < P_pad; k0 += 4 * KW) {
            fetch(k0);
            mma(a, b0, b1);
        }
    }
    if (wv > 0)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) red[wv - 1][r][c][lane] = acc[r][c];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            dbl4 v = acc[r][c];
            v += red[0][r][c][lane];
            v += red[1][r][c][lane];
            v += red[2][r][c][lane];
            const int col = 16 * c + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (col < nc) Zout[(int64_t)(row0 + 16 * r + 4 * e + lk) * nc + col] = v[e];
        }
}

void launch_kmatvec_skinny(Tracer *t, hipStream_t s, int P_pad, const double *K,
                           const double *Zin, double *Zout, int nc, double P) {
    trace_begin(t, "kernel_matvec", s);
    if (nc == 1)
        hipLaunchKernelGGL((k_kmatvec_lanes<1, 1>), dim3(P_pad / 4), dim3(256), 0, s, P_pad, K, Zin, Zout);
    else if (nc == 2)
        hipLaunchKernelGGL((k_kmatvec_lanes<2, 1>), dim3(P_pad / 4), dim3(256), 0, s, P_pad, K, Zin, Zout);
    else if (nc == 3)
        hipLaunchKernelGGL((k_kmatvec_lanes<3, 1>), dim3(P_pad / 4), dim3(256), 0, s, P_pad, K, Zin, Zout);
    else if (nc == 4)
        hipLaunchKernelGGL((k_kmatvec_lanes<4, 2>), dim3(P_pad / 8), dim3(256), 0, s, P_pad, K, Zin, Zout);
    else if (nc <= 16)
        hipLaunchKernelGGL((k_kmatvec_mfma<KMV_RT, 1, KMV_U, true>), dim3(P_pad / (16 * KMV_RT)), dim3(256), 0, s,
                           P_pad, K, Zin, Zout, nc);
    else
        hipLaunchKernelGGL((k_kmatvec_mfma<KMV_RT, 2, KMV_U / 2, false>), dim3(P_pad / (16 * KMV_RT)), dim3(256), 0,
                           s, P_pad, K, Zin, Zout, nc);
    trace_end(t, s, 2.0 * P * P * nc, 8.0 * (P * P + 2.0 * P * nc));
}

}  // namespace chi0
