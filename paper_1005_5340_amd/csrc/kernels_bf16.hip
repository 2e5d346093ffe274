// Split-BF16 x 3 matrix-core GEMM for the low-precision orbital transforms,
// and the conversions that prepare its operands.
//
// A value x (FP32) is carried as x_hi + x_lo with x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (round to nearest even), which keeps ~16 significant
// bits.  A product is formed as x_hi y_hi + x_hi y_lo + x_lo y_hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the lo*lo term is below
// the FP32 accumulation error and is dropped).
//
// v_mfma_f32_16x16x32_bf16, lane l = 0..63 (checked on gfx950 with a probe):
//   A (16 x 32): lane l holds A[l % 16][8*(l/16) + t], t = 0..7
//   B (32 x 16): lane l holds B[8*(l/16) + t][l % 16]
//   D (16 x 16): element r of lane l holds D[4*(l/16) + r][l % 16]
#include "common.h"

namespace chi0 {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int xcd_remap_b(int wid, int n) {
    const int q = n / 8, r = n % 8;
    const int x = wid % 8, local = wid / 8;
    return x * q + (x < r ? x : r) + local;
}

// C[M x N] (FP32) = A B with A given as BF16 hi/lo planes [M][lda] and B as
// BF16 hi/lo planes in k-blocks of 8: element (k, n) at ((k / 8) N + n) 8 + k % 8
// (k_split_kblk), so the 8 k of one column that an MFMA lane needs are one
// 16-byte load.  M % 64 == 0, K % 32 == 0 (per split), N masked.  blockIdx.y
// selects a K split as in the FP64 GEMM.
template <bool LORENTZ>
__global__ __launch_bounds__(256)
void k_bgemm3(int M, int N, int K, const uint16_t *__restrict__ Ahi, const uint16_t *__restrict__ Alo,
              int lda, const uint16_t *__restrict__ Bhi, const uint16_t *__restrict__ Blo,
              float *__restrict__ C, int ldc, int m_fastest, LorentzArgs la) {
    constexpr int BM = 64, BN = 64, BK = 32, PADK = BK + 8;
    __shared__ uint16_t Ash[2][BM][PADK], Asl[2][BM][PADK];
    __shared__ uint16_t Bsh[2][BN][PADK], Bsl[2][BN][PADK];   // transposed: [n][k]
    Ahi += (int64_t)blockIdx.y * K;
    Alo += (int64_t)blockIdx.y * K;
    Bhi += (int64_t)blockIdx.y * K * N;
    Blo += (int64_t)blockIdx.y * K * N;
    C += (int64_t)blockIdx.y * M * ldc;

    const int ntm = M / BM, ntn = (N + BN - 1) / BN;
    const int tile = xcd_remap_b(blockIdx.x, ntm * ntn);
    const int tm = m_fastest ? tile % ntm : tile / ntn;
    const int tn = m_fastest ? tile / ntm : tile % ntn;
    const int m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wm = wv % 2, wn = wv / 2;

    const int a_row = t / 4, a_k = (t % 4) * 8;          // 64 rows x 32 k, 8 per thread
    // B: thread t takes column n0 + (t % 64) and the k-block t / 64 (8 k): one
    // 16-byte load per plane, stored as one 16-byte row piece of the [n][k] tile.
    const int b_n = t & 63, b_kb = t >> 6;
    const uint16_t *ah = Ahi + (int64_t)(m0 + a_row) * lda + a_k;
    const uint16_t *al = Alo + (int64_t)(m0 + a_row) * lda + a_k;
    const bool b_ok = n0 + b_n < N;
    const int64_t boff = ((int64_t)b_kb * N + n0 + (b_ok ? b_n : 0)) * 8;

    uint4 rah, ral, rbh, rbl;
    auto load = [&](int kt) {
        rah = *reinterpret_cast<const uint4 *>(ah + kt * BK);
        ral = *reinterpret_cast<const uint4 *>(al + kt * BK);
        const int64_t o = boff + (int64_t)kt * (BK / 8) * N * 8;
        rbh = b_ok ? *reinterpret_cast<const uint4 *>(Bhi + o) : make_uint4(0, 0, 0, 0);
        rbl = b_ok ? *reinterpret_cast<const uint4 *>(Blo + o) : make_uint4(0, 0, 0, 0);
    };
    auto store = [&](int buf) {
        *reinterpret_cast<uint4 *>(&Ash[buf][a_row][a_k]) = rah;
        *reinterpret_cast<uint4 *>(&Asl[buf][a_row][a_k]) = ral;
        *reinterpret_cast<uint4 *>(&Bsh[buf][b_n][b_kb * 8]) = rbh;
        *reinterpret_cast<uint4 *>(&Bsl[buf][b_n][b_kb * 8]) = rbl;
    };

    flt4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    const int KT = K / BK;
    load(0);
    store(0);
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < KT) load(kt + 1);
        bf8 ahf[2], alf[2], bhf[2], blf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = wm * 32 + i * 16 + (lane & 15);
            ahf[i] = *reinterpret_cast<const bf8 *>(&Ash[cur][r][kq]);
            alf[i] = *reinterpret_cast<const bf8 *>(&Asl[cur][r][kq]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = wn * 32 + j * 16 + (lane & 15);
            bhf[j] = *reinterpret_cast<const bf8 *>(&Bsh[cur][c][kq]);
            blf[j] = *reinterpret_cast<const bf8 *>(&Bsl[cur][c][kq]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alf[i], bhf[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahf[i], blf[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahf[i], bhf[j], acc[i][j], 0, 0, 0);
            }
        if (kt + 1 < KT) store(cur ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
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
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                float v = acc[i][j][r];
                if (LORENTZ) {
                    const float other = __shfl_xor(v, 1);
                    const double D = la.Dlt[(int64_t)E * la.nv_pad + row];
                    const double d1 = w - D, d2 = w + D, e = la.eps;
                    const double s1 = 1.0 / (d1 * d1 + e * e), s2 = 1.0 / (d2 * d2 + e * e);
                    const double Lr = la.occ * (d1 * s1 - d2 * s2);
                    const double Li = la.occ * (-e * s1 + e * s2);
                    const double re = par ? other : v, im = par ? v : other;
                    v = (float)(par ? (re * Li + im * Lr) : (re * Lr - im * Li));
                }
                if (ok) C[(int64_t)row * ldc + col] = v;
            }
        }
    }
}

// Partial-product reduction of the FP32 GEMMs is shared with the FP32 path.
void launch_splitk_reduce_f32(Tracer *t, hipStream_t s, int M, int N, int S, const float *part,
                              float *C, int ldc, const LorentzArgs *la);

// B (FP32 [K][ldb], K % 8 == 0) -> hi/lo BF16 planes in k-blocks of 8 for
// k_bgemm3: thread (kb, n) reads the 8 rows of its block in column n
// (coalesced over n) and writes 16 bytes per plane.
__global__ __launch_bounds__(256)
void k_split_kblk(const float *__restrict__ B, int K, int N, int ldb, uint16_t *__restrict__ hi,
                  uint16_t *__restrict__ lo) {
    const int64_t total = (int64_t)(K / 8) * N;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int kb = (int)(idx / N), n = (int)(idx % N);
        const float *src = B + (int64_t)kb * 8 * ldb + n;
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int c = 0; c < 8; c += 2) {
            const float x0 = src[(int64_t)c * ldb], x1 = src[(int64_t)(c + 1) * ldb];
            const uint16_t h0 = f2bf(x0), h1 = f2bf(x1);
            const uint16_t l0 = f2bf(x0 - bf2f(h0)), l1 = f2bf(x1 - bf2f(h1));
            hw[c / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
            lw[c / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
        }
        reinterpret_cast<uint4 *>(hi)[idx] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        reinterpret_cast<uint4 *>(lo)[idx] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
}

void launch_bgemm3(Tracer *t, hipStream_t s, const char *name, int M, int N, int K,
                   const uint16_t *Ahi, const uint16_t *Alo, int lda, const float *B, int ldb,
                   uint16_t *Bhi, uint16_t *Blo, float *C, int ldc, double flops, double bytes,
                   const LorentzArgs *la, void *scratch, size_t scratch_bytes) {
    {   // B split once into the k-blocked hi/lo planes
        int64_t blocks = ((int64_t)(K / 8) * N + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        trace_begin(t, "bf16_split", s);
        hipLaunchKernelGGL(k_split_kblk, dim3((unsigned)blocks), dim3(256), 0, s, B, K, N, ldb, Bhi, Blo);
        trace_end(t, s, 0.0, 8.0 * (double)K * N);
    }
    const int tiles = (M / 64) * ((N + 63) / 64);
    const int KT = K / 32;
    int S = 1;
    while (scratch && S < 16 && tiles * S < 1024 && KT % (2 * S) == 0 && KT / (2 * S) >= 4 &&
           (size_t)(2 * S) * M * (size_t)N * sizeof(float) <= scratch_bytes)
        S *= 2;
    const int m_fastest = (M / 64) <= ((N + 63) / 64);
    LorentzArgs none{};
    trace_begin(t, name, s);
    if (S == 1) {
        if (la)
            hipLaunchKernelGGL(k_bgemm3<true>, dim3(tiles, 1), dim3(256), 0, s, M, N, K, Ahi, Alo, lda,
                               (const uint16_t *)Bhi, (const uint16_t *)Blo, C, ldc, m_fastest, *la);
        else
            hipLaunchKernelGGL(k_bgemm3<false>, dim3(tiles, 1), dim3(256), 0, s, M, N, K, Ahi, Alo, lda,
                               (const uint16_t *)Bhi, (const uint16_t *)Blo, C, ldc, m_fastest, none);
        trace_end(t, s, flops, bytes);
        return;
    }
    float *part = static_cast<float *>(scratch);
    hipLaunchKernelGGL(k_bgemm3<false>, dim3(tiles, S), dim3(256), 0, s, M, N, K / S, Ahi, Alo, lda,
                       (const uint16_t *)Bhi, (const uint16_t *)Blo, part, N, m_fastest, none);
    trace_end(t, s, flops, bytes);
    launch_splitk_reduce_f32(t, s, M, N, S, part, C, ldc, la);
}

// ------------------------------------------------------------- conversions
__global__ __launch_bounds__(256) void k_to_f32(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] = (float)x[i];
}

__global__ __launch_bounds__(256) void k_split_bf16(const double *__restrict__ x, uint16_t *__restrict__ hi,
                                                    uint16_t *__restrict__ lo, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float f = (float)x[i];
        const uint16_t h = f2bf(f);
        hi[i] = h;
        lo[i] = f2bf(f - bf2f(h));
    }
}

void launch_to_f32(hipStream_t s, const double *x, float *y, int64_t n) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n);
}

void launch_split_bf16(hipStream_t s, const double *x, uint16_t *hi, uint16_t *lo, int64_t n) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (n > 0) hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)blocks), dim3(256), 0, s, x, hi, lo, n);
}

}  // namespace chi0
