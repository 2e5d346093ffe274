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

// Column tile of the vertex kernels: a power of two <= 64 covering nc.
static int vertex_jt(int nc) {
    int jt = 1;
    while (jt < nc && jt < 64) jt <<= 1;
    return jt;
}

// (a) dV[(ent_k + ab)][j] = sum_i Vp[k][i][ab] * Z[pidx[k][i]][j]
__global__ __launch_bounds__(256)
void k_vertex_gather(BlockMapDev bm, const double *__restrict__ Z, double *__restrict__ dV,
                     int nc, int jt) {
    constexpr int R = 4;
    const int k = blockIdx.x;
    const int t = threadIdx.x, jj = t % jt, grp = t / jt, G = 256 / jt;
    const int j = blockIdx.y * jt + jj;
    const int nAB = bm.blk_na[k] * bm.blk_nb[k];
    const int np = bm.blk_nprod[k];
    const double *Vk = bm.Vp + bm.blk_vstart[k];
    const int32_t *pk = bm.pidx + bm.blk_pstart[k];
    const int64_t ent = bm.blk_ent[k];
    const bool valid = j < nc;
    for (int ab0 = grp; ab0 < nAB; ab0 += G * R) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int i = 0; i < np; ++i) {
            const double zv = valid ? Z[(int64_t)pk[i] * nc + j] : 0.0;
            const double *vi = Vk + (int64_t)i * nAB;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ab = ab0 + r * G;
                if (ab < nAB) acc[r] += vi[ab] * zv;
            }
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ab = ab0 + r * G;
                if (ab < nAB) dV[(ent + ab) * nc + j] = acc[r];
            }
        }
    }
}

void launch_vertex_gather(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_blk,
                          const double *Z, double *dV, int nc, const WorkSizes &ws) {
    const int jt = vertex_jt(nc);
    dim3 grid(n_blk, (nc + jt - 1) / jt);
    trace_begin(t, "vertex_gather", s);
    hipLaunchKernelGGL(k_vertex_gather, grid, dim3(256), 0, s, bm, Z, dV, nc, jt);
    trace_end(t, s, 2.0 * ws.sum_s2 * nc, 8.0 * (ws.sum_s2 + ws.P * nc + ws.nnzB * nc));
}

// (d), first pass: part[pstart_k + i][j] = sum_ab Vp[k][i][ab] * W[(ent_k + ab)][j]
constexpr int JTD = 32;             // max columns per workgroup (LDS: NB_MAX^2 x JTD doubles)
__global__ __launch_bounds__(256)
void k_vertex_contract(BlockMapDev bm, const double *__restrict__ W, double *__restrict__ part,
                       int nc, int jt) {
    __shared__ double Ws[NB_MAX * NB_MAX * JTD];
    const int k = blockIdx.x;
    const int t = threadIdx.x, jj = t % jt, grp = t / jt, G = 256 / jt;
    const int j0 = blockIdx.y * jt, j = j0 + jj;
    const int nAB = bm.blk_na[k] * bm.blk_nb[k];
    const int np = bm.blk_nprod[k];
    const int64_t ent = bm.blk_ent[k];
    for (int idx = t; idx < nAB * jt; idx += 256) {
        const int ab = idx / jt, c = idx % jt;
        Ws[ab * jt + c] = (j0 + c < nc) ? W[(ent + ab) * nc + j0 + c] : 0.0;
    }
    __syncthreads();
    if (j >= nc) return;
    const double *Vk = bm.Vp + bm.blk_vstart[k];
    const int64_t p0 = bm.blk_pstart[k];
    for (int i = grp; i < np; i += G) {
        const double *vi = Vk + (int64_t)i * nAB;
        double acc = 0.0;
        for (int ab = 0; ab < nAB; ++ab) acc += vi[ab] * Ws[ab * jt + jj];
        part[(p0 + i) * nc + j] = acc;
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
                            const double *W, double *part, double *Y, int nc, const WorkSizes &ws) {
    int jt = vertex_jt(nc);
    if (jt > JTD) jt = JTD;
    dim3 grid(n_blk, (nc + jt - 1) / jt);
    trace_begin(t, "vertex_contract", s);
    hipLaunchKernelGGL(k_vertex_contract, grid, dim3(256), 0, s, bm, W, part, nc, jt);
    trace_end(t, s, 2.0 * ws.sum_s2 * nc, 8.0 * (ws.sum_s2 + ws.nnzB * nc + ws.npart * nc));
    const int64_t n = (int64_t)P * nc;
    trace_begin(t, "vertex_reduce", s);
    hipLaunchKernelGGL(k_vertex_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       bm, P, part, Y, nc);
    trace_end(t, s, ws.npart * nc, 8.0 * (ws.npart * nc + ws.P * nc));
}

}  // namespace chi0
