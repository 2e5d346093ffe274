// Kernels of the learned GMRES warm start: a reduced basis U of training
// solutions and a small network c(w) so that x0 = U c(w).
//
// The network is a 3-layer perceptron on Fourier features of the frequency,
// trained by full-batch Adam.  Weights and activations are FP32; every
// matrix product rounds its operands to BF16 (round to nearest even) and
// accumulates in FP32 on v_mfma_f32_16x16x32_bf16 (lane layout: A[l%16][8(l/16)+t],
// B[8(l/16)+t][l%16], D[4(l/16)+r][l%16]).
#include "common.h"

namespace chi0 {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf_m(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// C[M x N] = op(A) op(B) with op(A)[m][k] = A[m*sam + k*sak] and
// op(B)[k][n] = B[k*sbk + n*sbn]; M, N % 16 == 0, K % 32 == 0.  One
// wavefront per 16 x 16 output tile, operands read straight from global.
__global__ __launch_bounds__(256)
void k_mlp_gemm(int M, int N, int K, const float *__restrict__ A, int sam, int sak,
                const float *__restrict__ B, int sbk, int sbn, float *__restrict__ C, int ldc) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int mt = M / 16;
    if (w >= mt * (N / 16)) return;
    const int tm = w % mt, tn = w / mt;
    const int row = tm * 16 + (lane & 15), col = tn * 16 + (lane & 15), kq = 8 * (lane >> 4);
    flt4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        u16x8 ua, ub;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = k0 + kq + t;
            ua[t] = f2bf_m(A[(int64_t)row * sam + (int64_t)k * sak]);
            ub[t] = f2bf_m(B[(int64_t)k * sbk + (int64_t)col * sbn]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ua),
                                                     __builtin_bit_cast(bf8, ub), acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        C[(int64_t)(tm * 16 + 4 * (lane >> 4) + r) * ldc + col] = acc[r];
}

void launch_mlp_gemm(hipStream_t s, int M, int N, int K, const float *A, int sam, int sak,
                     const float *B, int sbk, int sbn, float *C, int ldc) {
    const int waves = (M / 16) * (N / 16);
    hipLaunchKernelGGL(k_mlp_gemm, dim3((waves + 3) / 4), dim3(256), 0, s, M, N, K, A, sam, sak, B,
                       sbk, sbn, C, ldc);
}

// phi[i][2(k-1)] = sin(k pi w_i / scale), phi[i][2(k-1)+1] = cos(k pi w_i / scale), k = 1..nf;
// rows i >= n (batch padding) are zero.
__global__ void k_features(int n, int n_pad, const double *__restrict__ omega, int nf, double scale,
                           float *__restrict__ phi) {
    const int i = blockIdx.x, k = threadIdx.x;   // k < nf
    if (k >= nf) return;
    float sv = 0.f, cv = 0.f;
    if (i < n) {
        const double a = (k + 1) * 3.14159265358979323846 * omega[i] / scale;
        sv = (float)sin(a);
        cv = (float)cos(a);
    }
    phi[(int64_t)i * 2 * nf + 2 * k] = sv;
    phi[(int64_t)i * 2 * nf + 2 * k + 1] = cv;
    (void)n_pad;
}

void launch_features(hipStream_t s, int n, int n_pad, const double *omega, int nf, double scale,
                     float *phi) {
    hipLaunchKernelGGL(k_features, dim3(n_pad), dim3(64), 0, s, n, n_pad, omega, nf, scale, phi);
}

// Z[m][n] = act(Z[m][n] + bias[n]); act 1 = tanh, 0 = identity.
__global__ void k_bias_act(int M, int N, float *__restrict__ Z, const float *__restrict__ bias, int act) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    float v = Z[i] + bias[i % N];
    Z[i] = act ? tanhf(v) : v;
}

void launch_bias_act(hipStream_t s, int M, int N, float *Z, const float *bias, int act) {
    const int64_t n = (int64_t)M * N;
    hipLaunchKernelGGL(k_bias_act, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M, N, Z, bias, act);
}

// Mean squared error over the first n_rows rows and n_cols columns; dOut =
// d loss / d out (zero in padding).  Single workgroup, fixed-order reduction.
__global__ __launch_bounds__(256)
void k_mse(int M, int N, int n_rows, int n_cols, const float *__restrict__ out,
           const float *__restrict__ tgt, float *__restrict__ dout, float *__restrict__ loss) {
    __shared__ float sh[256];
    const float scale = 1.f / ((float)n_rows * (float)n_cols);
    float acc = 0.f;
    for (int i = threadIdx.x; i < M * N; i += 256) {
        const int r = i / N, c = i % N;
        float d = 0.f;
        if (r < n_rows && c < n_cols) d = out[i] - tgt[i];
        acc += d * d;
        dout[i] = 2.f * d * scale;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] * scale;
}

void launch_mse(hipStream_t s, int M, int N, int n_rows, int n_cols, const float *out, const float *tgt,
                float *dout, float *loss) {
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, M, N, n_rows, n_cols, out, tgt, dout, loss);
}

// dZ = dH * (1 - H^2) (tanh derivative), in place on dH.
__global__ void k_tanh_back(int64_t n, const float *__restrict__ H, float *__restrict__ dH) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dH[i] *= 1.f - H[i] * H[i];
}

void launch_tanh_back(hipStream_t s, int64_t n, const float *H, float *dH) {
    hipLaunchKernelGGL(k_tanh_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, H, dH);
}

// db[n] = sum_m dZ[m][n] (fixed order).
__global__ void k_colsum(int M, int N, const float *__restrict__ dZ, float *__restrict__ db) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= N) return;
    float a = 0.f;
    for (int m = 0; m < M; ++m) a += dZ[(int64_t)m * N + c];
    db[c] = a;
}

void launch_colsum(hipStream_t s, int M, int N, const float *dZ, float *db) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, M, N, dZ, db);
}

// Adam with bias correction (Kingma & Ba), step t >= 1.
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, int t) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t)), vh = vi / (1.f - powf(b2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

void launch_adam(hipStream_t s, int64_t n, float *p, const float *g, float *m, float *v, float lr,
                 float b1, float b2, float eps, int t) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, g, m, v, lr, b1,
                       b2, eps, t);
}

// G[i][j] = <S_i | S_j> (Hermitian Gram matrix of n complex vectors), one wavefront per entry.
__global__ __launch_bounds__(256)
void k_gram(int n, const double *__restrict__ S, int64_t stride, int P, double *__restrict__ G) {
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= n * n) return;
    const int i = e / n, j = e % n;
    const double2 *a = reinterpret_cast<const double2 *>(S + (int64_t)i * stride);
    const double2 *b = reinterpret_cast<const double2 *>(S + (int64_t)j * stride);
    double re = 0.0, im = 0.0;
    for (int mu = lane; mu < P; mu += 64) {
        const double2 x = a[mu], y = b[mu];
        re += x.x * y.x + x.y * y.y;
        im += x.x * y.y - x.y * y.x;
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if (lane == 0) {
        G[2 * e] = re;
        G[2 * e + 1] = im;
    }
}

void launch_gram(hipStream_t s, int n, const double *S, int64_t stride, int P, double *G) {
    hipLaunchKernelGGL(k_gram, dim3((n * n + 3) / 4), dim3(256), 0, s, n, S, stride, P, G);
}

// U[k][mu] = sum_t S[t][mu] Wc[t][k]  (complex; S [n][stride], Wc [n][r], U [r][stride])
__global__ __launch_bounds__(256)
void k_basis(int n, int r, const double *__restrict__ S, int64_t stride, int P,
             const double *__restrict__ Wc, double *__restrict__ U) {
    const int mu = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y;
    if (mu >= P) return;
    double re = 0.0, im = 0.0;
    for (int t = 0; t < n; ++t) {
        const double2 x = reinterpret_cast<const double2 *>(S + (int64_t)t * stride)[mu];
        const double wr = Wc[2 * (t * r + k)], wi = Wc[2 * (t * r + k) + 1];
        re += x.x * wr - x.y * wi;
        im += x.x * wi + x.y * wr;
    }
    reinterpret_cast<double2 *>(U + (int64_t)k * stride)[mu] = make_double2(re, im);
}

void launch_basis(hipStream_t s, int n, int r, const double *S, int64_t stride, int P, const double *Wc,
                  double *U) {
    hipLaunchKernelGGL(k_basis, dim3((P + 255) / 256, r), dim3(256), 0, s, n, r, S, stride, P, Wc, U);
}

// x[jobs[q].slot] = U c with c_k = (mean + std * out)[2k] + i (mean + std * out)[2k+1]
// for row q of the network output.  U [r][ustride], x [*][xstride] (complex).
__global__ __launch_bounds__(256)
void k_ws_apply(const Job *__restrict__ jobs, const float *__restrict__ out, int ldo,
                const float *__restrict__ mean, const float *__restrict__ sdev, int r,
                const double *__restrict__ U, int64_t ustride, double *__restrict__ x,
                int64_t xstride, int P) {
    extern __shared__ double cs[];
    const int q = blockIdx.y, t = threadIdx.x;
    for (int i = t; i < 2 * r; i += 256) cs[i] = (double)mean[i] + (double)sdev[i] * (double)out[(int64_t)q * ldo + i];
    __syncthreads();
    const int mu = blockIdx.x * 256 + t;
    if (mu >= P) return;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < r; ++k) {
        const double2 u = reinterpret_cast<const double2 *>(U + (int64_t)k * ustride)[mu];
        re += u.x * cs[2 * k] - u.y * cs[2 * k + 1];
        im += u.x * cs[2 * k + 1] + u.y * cs[2 * k];
    }
    reinterpret_cast<double2 *>(x + (int64_t)jobs[q].slot * xstride)[mu] = make_double2(re, im);
}

void launch_ws_apply(hipStream_t s, const Job *jobs, int n, const float *out, int ldo, const float *mean,
                     const float *sdev, int r, const double *U, int64_t ustride, double *x,
                     int64_t xstride, int P) {
    hipLaunchKernelGGL(k_ws_apply, dim3((P + 255) / 256, n), dim3(256), (size_t)2 * r * sizeof(double), s,
                       jobs, out, ldo, mean, sdev, r, U, ustride, x, xstride, P);
}

// Zero start after a rejected warm start: x = 0, v0 = b/||b||, g0 = ||b||.
__global__ __launch_bounds__(256)
void k_reset_slots(const Job *__restrict__ jobs, SlotsDev sl, int P) {
    __shared__ double sh[4];
    const int q = blockIdx.x, t = threadIdx.x;
    const int s = jobs[q].slot;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    double2 *x = reinterpret_cast<double2 *>(sl.x + s * vlen);
    const double2 *b = reinterpret_cast<const double2 *>(sl.b + s * vlen);
    double2 *v0 = reinterpret_cast<double2 *>(sl.V + s * sl.vstride);
    double ss = 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = b[mu];
        ss += a.x * a.x + a.y * a.y;
        x[mu] = make_double2(0.0, 0.0);
    }
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
    if ((t & 63) == 0) sh[t >> 6] = ss;
    __syncthreads();
    const double nrm = sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
    const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int mu = t; mu < P; mu += 256) {
        const double2 a = b[mu];
        v0[mu] = make_double2(a.x * sc, a.y * sc);
    }
    if (t == 0) {
        sl.g[(int64_t)s * (sl.m + 1) * 2] = nrm;
        sl.g[(int64_t)s * (sl.m + 1) * 2 + 1] = 0.0;
    }
}

void launch_reset_slots(hipStream_t s, const Job *jobs, int n, const SlotsDev &sl, int P) {
    hipLaunchKernelGGL(k_reset_slots, dim3(n), dim3(256), 0, s, jobs, sl, P);
}

// Copy the solution of finished points to out[point][P_pad] (training data).
__global__ __launch_bounds__(256)
void k_store_x(const Job *__restrict__ jobs, SlotsDev sl, int P, double *__restrict__ out) {
    const int q = blockIdx.y, mu = blockIdx.x * 256 + threadIdx.x;
    if (mu >= P) return;
    const int64_t vlen = (int64_t)sl.P_pad * 2;
    reinterpret_cast<double2 *>(out + (int64_t)jobs[q].j * vlen)[mu] =
        reinterpret_cast<const double2 *>(sl.x + jobs[q].slot * vlen)[mu];
}

void launch_store_x(hipStream_t s, const Job *jobs, int n, const SlotsDev &sl, int P, double *out) {
    hipLaunchKernelGGL(k_store_x, dim3((P + 255) / 256, n), dim3(256), 0, s, jobs, sl, P, out);
}

}  // namespace chi0
