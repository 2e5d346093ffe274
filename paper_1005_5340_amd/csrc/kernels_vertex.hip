// Vertex kernels of the matrix-free chi0 product (Sec. 4.2, Table t:flops
// steps 2 and 5): the contraction of the product-space vector with the
// sparse vertex, dV_ab = sum_mu z_mu V_mu^{ab}, and its transpose, the
// projection n_mu = sum_ab V_mu^{ab} W_ab.
//
// The vertex is stored per atom-pair block (A, B) as a panel holding, for
// every product whose support covers (A, B), its n_A x n_B sub-block.  Both
// kernels walk one block per workgroup, so every vertex element is read
// once per call and no atomics are needed: the projection writes one
// partial sum per (block, product) and a second pass adds the (at most 4)
// partials of each product in a fixed order.
#include "common.h"

namespace chi0 {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma16(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Both vertex kernels are small GEMMs per atom-pair block on the FP64 matrix
// cores (16x16x4; lane l holds A[l%16][l/16], B[l/16][l%16] and returns
// D[4r + l/16][l%16]).  A workgroup owns one block and VC 16-column MFMA
// blocks; wave w owns the 16-row blocks w, w+4, w+8, w+12 of the block's
// output.  Each round issues the operand loads of KU k-steps before their
// MFMAs, so a round costs about one memory latency and the longest block
// (a diagonal block (A, A), which carries every product that involves atom
// A) runs few rounds.  The narrow shapes (VC = 1, 2) hold fewer
// accumulators, which leaves registers for 8 k-steps' loads per round
// instead of 4 at two waves per SIMD.  Every shape accumulates each output
// over k in the same order, so all of them give bit-identical results.
constexpr int VRB = 4;     // 16-row MFMA blocks per wave (rows <= 256 = NB_MAX^2)
constexpr int PCH = 256;   // product ids staged in LDS per chunk

// (a) dV[(ent_k + ab)][j] = sum_i Vp[k][i][ab] * Z[pidx[k][i]][j]
//     rows = ab (n_A n_B), K = the block's products, columns = j.
template <int VC, int KU>
__global__ __launch_bounds__(256)
void k_vertex_gather(BlockMapDev bm, const double *__restrict__ Z, double *__restrict__ dV, int nc) {
    __shared__ int32_t ps[PCH];
    const int k = blockIdx.x, j0 = blockIdx.y * 16 * VC;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int nAB = bm.blk_na[k] * bm.blk_nb[k];
    const int np = bm.blk_nprod[k];
    const double *Vk = bm.Vp + bm.blk_vstart[k];
    const int32_t *pk = bm.pidx + bm.blk_pstart[k];
    const int64_t ent = bm.blk_ent[k];
    const int nrb = (nAB + 15) / 16, ncb = min(VC, (nc - j0 + 15) / 16);
    const int lr = lane & 15, lk = lane >> 4;

    dbl4 acc[VRB][VC];
#pragma unroll
    for (int r = 0; r < VRB; ++r)
#pragma unroll
        for (int c = 0; c < VC; ++c) acc[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int c0 = 0; c0 < np; c0 += PCH) {
        const int cn = min(PCH, np - c0);
        __syncthreads();
        if (t < cn) ps[t] = pk[c0 + t];
        __syncthreads();
        // KU k-steps of 4 products per round: all their loads are issued
        // before their MFMAs; k-steps past the chunk's end are skipped
        for (int i0 = 0; i0 < cn; i0 += 4 * KU) {
            double a[KU][VRB], b[KU][VC];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int kk = i0 + 4 * u + lk;
                const bool kv = kk < cn;
                const int64_t zrow = kv ? (int64_t)ps[kk] * nc : 0;
#pragma unroll
                for (int r = 0; r < VRB; ++r) {
                    const int row = (wv + 4 * r) * 16 + lr;
                    a[u][r] = (kv && row < nAB) ? Vk[(int64_t)(c0 + kk) * nAB + row] : 0.0;
                }
#pragma unroll
                for (int c = 0; c < VC; ++c) {
                    const int j = j0 + c * 16 + lr;
                    b[u][c] = (kv && j < nc) ? Z[zrow + j] : 0.0;
                }
            }
#pragma unroll
            for (int r = 0; r < VRB; ++r) {
                if (wv + 4 * r >= nrb) continue;
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    if (i0 + 4 * u >= cn) continue;
#pragma unroll
                    for (int c = 0; c < VC; ++c)
                        if (c < ncb) acc[r][c] = mfma16(a[u][r], b[u][c], acc[r][c]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < VRB; ++r) {
        if (wv + 4 * r >= nrb) continue;
#pragma unroll
        for (int c = 0; c < VC; ++c) {
            const int j = j0 + c * 16 + lr;
            if (c >= ncb || j >= nc) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = (wv + 4 * r) * 16 + 4 * e + lk;
                if (row < nAB) dV[(ent + row) * nc + j] = acc[r][c][e];
            }
        }
    }
}

// 16-column MFMA blocks per workgroup for nc columns: 1 up to 16 columns,
// 2 up to 32, else 4
static int vertex_vc(int nc) { return nc <= 16 ? 1 : nc <= 32 ? 2 : 4; }

void launch_vertex_gather(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_blk,
                          const double *Z, double *dV, int nc, const WorkSizes &ws) {
    const int vc = vertex_vc(nc);
    dim3 grid(n_blk, (nc + 16 * vc - 1) / (16 * vc));
    trace_begin(t, "vertex_gather", s);
    if (vc == 1)
        hipLaunchKernelGGL((k_vertex_gather<1, 8>), grid, dim3(256), 0, s, bm, Z, dV, nc);
    else if (vc == 2)
        hipLaunchKernelGGL((k_vertex_gather<2, 8>), grid, dim3(256), 0, s, bm, Z, dV, nc);
    else
        hipLaunchKernelGGL((k_vertex_gather<4, 4>), grid, dim3(256), 0, s, bm, Z, dV, nc);
    trace_end(t, s, 2.0 * ws.sum_s2 * nc, 8.0 * (ws.sum_s2 + ws.P * nc + ws.nnzB * nc));
}

// (d), first pass: part[pstart_k + i][j] = sum_ab Vp[k][i][ab] * W[(ent_k + ab)][j]
//     rows = the block's products, K = ab, columns = j.
// A workgroup whose products fit one 16-row MFMA block (every off-diagonal
// block: it carries only its pair's bilocal products) would leave three of
// its four waves idle through the whole ab range; there the waves take
// turns over the rounds of k-steps instead (wave w the rounds w, w+4, ...)
// and their partial sums are added in wave order through LDS.  Whether a
// workgroup splits depends on the block alone, so every column shape still
// gives the same results.
template <int VC, int KU>
__global__ __launch_bounds__(256)
void k_vertex_contract(BlockMapDev bm, const double *__restrict__ W, double *__restrict__ part,
                       int nc) {
    __shared__ dbl4 red[3][VC][64];   // partial sums of waves 1-3 when the k range is split
    const int k = blockIdx.x, j0 = blockIdx.y * 16 * VC, rb0 = blockIdx.z * 4 * VRB;
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nAB = bm.blk_na[k] * bm.blk_nb[k];
    const int np = bm.blk_nprod[k];
    const double *Vk = bm.Vp + bm.blk_vstart[k];
    const int64_t ent = bm.blk_ent[k];
    const int64_t p0 = bm.blk_pstart[k];
    const int nrb = (np + 15) / 16, ncb = min(VC, (nc - j0 + 15) / 16);
    if (rb0 >= nrb) return;
    const int lr = lane & 15, lk = lane >> 4;
    const bool split = nrb - rb0 == 1;          // uniform over the workgroup
    const int rw = split ? 0 : wv;              // this wave's first row block (past rb0)
    const int kstep = (split ? 4 : 1) * 4 * KU; // ab advanced per round of this wave

    dbl4 acc[VRB][VC];
#pragma unroll
    for (int r = 0; r < VRB; ++r)
#pragma unroll
        for (int c = 0; c < VC; ++c) acc[r][c] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int a0 = (split ? wv : 0) * 4 * KU; a0 < nAB; a0 += kstep) {
        double a[KU][VRB], b[KU][VC];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int kk = a0 + 4 * u + lk;
            const bool kv = kk < nAB;
#pragma unroll
            for (int r = 0; r < VRB; ++r) {
                const int i = (rb0 + rw + 4 * r) * 16 + lr;
                a[u][r] = (kv && i < np) ? Vk[(int64_t)i * nAB + kk] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < VC; ++c) {
                const int j = j0 + c * 16 + lr;
                b[u][c] = (kv && j < nc) ? W[(ent + kk) * nc + j] : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < VRB; ++r) {
            if (rb0 + rw + 4 * r >= nrb) continue;
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                if (a0 + 4 * u >= nAB) continue;
#pragma unroll
                for (int c = 0; c < VC; ++c)
                    if (c < ncb) acc[r][c] = mfma16(a[u][r], b[u][c], acc[r][c]);
            }
        }
    }
    if (split) {
        if (wv > 0)
#pragma unroll
            for (int c = 0; c < VC; ++c) red[wv - 1][c][lane] = acc[0][c];
        __syncthreads();
        if (wv > 0) return;
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int c = 0; c < VC; ++c) acc[0][c] += red[w][c][lane];
    }
#pragma unroll
    for (int r = 0; r < VRB; ++r) {
        if (rb0 + rw + 4 * r >= nrb) continue;
#pragma unroll
        for (int c = 0; c < VC; ++c) {
            const int j = j0 + c * 16 + lr;
            if (c >= ncb || j >= nc) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = (rb0 + rw + 4 * r) * 16 + 4 * e + lk;
                if (i < np) part[(p0 + i) * nc + j] = acc[r][c][e];
            }
        }
    }
}

// (d), second pass: Y[mu][j] = sum over the (block, slot) entries of mu, in order.
__global__ __launch_bounds__(256)
void k_vertex_reduce(BlockMapDev bm, int P, const double *__restrict__ part,
                     double *__restrict__ Y, int nc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)P * nc) return;
    const int mu = (int)(idx / nc), j = (int)(idx % nc);
    double acc = 0.0;
    for (int64_t s = bm.prod_pstart[mu]; s < bm.prod_pstart[mu + 1]; ++s)
        acc += part[bm.prod_plist[s] * nc + j];
    Y[idx] = acc;
}

void launch_vertex_contract(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_blk, int P,
                            const double *W, double *part, double *Y, int nc, const WorkSizes &ws,
                            int max_nprod) {
    const int rgroups = ((max_nprod + 15) / 16 + 4 * VRB - 1) / (4 * VRB);
    const int vc = vertex_vc(nc);
    dim3 grid(n_blk, (nc + 16 * vc - 1) / (16 * vc), rgroups);
    trace_begin(t, "vertex_contract", s);
    if (vc == 1)
        hipLaunchKernelGGL((k_vertex_contract<1, 8>), grid, dim3(256), 0, s, bm, W, part, nc);
    else if (vc == 2)
        hipLaunchKernelGGL((k_vertex_contract<2, 8>), grid, dim3(256), 0, s, bm, W, part, nc);
    else
        hipLaunchKernelGGL((k_vertex_contract<4, 4>), grid, dim3(256), 0, s, bm, W, part, nc);
    trace_end(t, s, 2.0 * ws.sum_s2 * nc, 8.0 * (ws.sum_s2 + ws.nnzB * nc + ws.npart * nc));
    const int64_t n = (int64_t)P * nc;
    trace_begin(t, "vertex_reduce", s);
    hipLaunchKernelGGL(k_vertex_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       bm, P, part, Y, nc);
    trace_end(t, s, ws.npart * nc, 8.0 * (ws.npart * nc + ws.P * nc));
}

}  // namespace chi0
