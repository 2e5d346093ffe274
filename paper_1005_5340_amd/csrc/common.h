// Internal declarations shared by the HIP translation units of libchi0.
//
// Device data layout (all FP64; "pad" sizes are multiples of the tile sizes
// and the padding is kept at zero so no kernel needs edge checks along it):
//   Xo   [N_pad][No_pad]   occupied columns of X, row = atomic orbital
//   Xv   [N_pad][Nv_pad]   virtual columns of X
//   Xvt  [Nv_pad][N_pad]   transpose of Xv
//   Dlt  [No_pad][Nv_pad]  transition energies e_F - e_E (padding = 1)
//   K    [P_pad][P_pad]    kernel matrix
//   Vp   per atom-pair block k=(A,B): the sub-blocks V_mu[A-part][B-part] of
//        every product mu whose support covers (A,B), each n_A x n_B row-major
//
// A batch of nb complex right-hand sides is carried as nc = 2*nb real
// columns (column 2r = real part, 2r+1 = imaginary part of RHS r).  Operator
// buffers are [rows][nc].  The orbital-transform intermediates index their
// long dimension by m = E*nc + j (occupied state E, column j):
//   dV, W [nnzB][nc]             block-sparse, entry (k, a, b) -> row ent(k)+a*n_B+b
//   Tt, Ut [N_pad][No_pad*nc]    Tt[b][m] = (X_occ^T dV)[E][b] of column j
//   at    [Nv_pad][No_pad*nc]    at[F][m] = (X_occ^T dV X_virt)[E][F], then scaled
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>

namespace chi0 {

constexpr int TILE = 64;     // M/N tile of the dense GEMMs, E tile of the gathered ones
constexpr int NB_MAX = 16;   // maximum orbitals per atom (a vertex block's n_A n_B rows <= 256)
constexpr int GEMM_VARIANTS = 6;   // tile shapes of the dense GEMM (see GemmTuner)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------- kernel timing
// Every launch goes through launch_begin/launch_end so that per-kernel
// durations can be accumulated with HIP events when tracing is enabled.
struct Tracer;
void trace_begin(Tracer *t, const char *name, hipStream_t s);
void trace_end(Tracer *t, hipStream_t s, double flops = 0.0, double bytes = 0.0);

// Unpadded sizes for the algorithmic work counts of the tracer.
struct WorkSizes {
    double N = 0, No = 0, Nv = 0, P = 0, nnzB = 0, sum_s2 = 0, npart = 0;
};

// Frequency factor of (b2)+(c): GEMM column n <-> (E, j) with E = n / ncp,
// j = n % ncp; columns 2r and 2r+1 hold Re and Im of RHS r; GEMM row = virtual F.
struct LorentzArgs {
    const double *Dlt;   // [No_pad][Nv_pad]
    const double *omega; // [ncp/2]
    int nv_pad;
    int ncp;
    double eps;
    double occ;
};

// -------------------------------------------------------------- chi0 blocks
struct BlockMapDev {
    // per atom-pair block k (n_blk of them)
    const int32_t *blk_nprod;     // products covering the block
    const int64_t *blk_pstart;    // start of the block's entries in pidx / part
    const int64_t *blk_vstart;    // start of the block's vertex panel in Vp (doubles)
    const int64_t *blk_ent;       // first entry row of the block in dV / W
    const int32_t *blk_na;        // n_A
    const int32_t *blk_nb;        // n_B
    const int32_t *pidx;          // [sum nprod] product of each (block, slot)
    const double *Vp;             // vertex panels
    // per column atom B: gathered rows (A, a) over the blocks (A, B)
    const int32_t *col_gstart;    // [n_atoms+1] start of atom B's gathered rows
    const int32_t *g_xrow;        // [n_g] global orbital a of the row
    const int64_t *g_ent;         // [n_g] entry row of (k(A,B), a, b=0) in dV / W
    const int32_t *atom_off;      // [n_atoms+1] orbital offsets
    // per product: positions of its (block, slot) pairs in part
    const int64_t *prod_pstart;   // [P+1]
    const int64_t *prod_plist;    // [sum]
    int nb_max;                   // largest number of orbitals on one atom
};

// ------------------------------------------------------------ launch wrappers
// (a) dV = sum_mu z_mu V_mu, per block.
void launch_vertex_gather(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_blk,
                          const double *Z, double *dV, int nc, const WorkSizes &ws);
// (d) n_mu = <V_mu, W>: per-block partial sums, then the sum over each product's blocks.
// max_nprod = largest number of products covering one block.
void launch_vertex_contract(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_blk, int P,
                            const double *W, double *part, double *Y, int nc, const WorkSizes &ws,
                            int max_nprod);
// (b1) Tt = X_occ^T dV (gathered MFMA GEMM over the block pattern).
void launch_occ_transform(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms,
                          const double *Xo, int no_pad, const double *dV, double *Tt,
                          int nc, const WorkSizes &ws);
// (b4) W = X_occ Ut restricted to the block pattern; the sum over occupied
// states runs over E < no_sum (a multiple of 16, at most no_pad).
void launch_occ_back(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms, int max_rows,
                     const double *Xo, int no_pad, int no_sum, const double *Ut, double *W, int nc,
                     const WorkSizes &ws);
// Tile-shape autotuner of the dense GEMMs (one per context).  The first call
// of a GEMM whose (name, M, K, split count, N within a half octave) has not
// been seen times every tile variant valid for it (HIP events, one warm and
// the best of three timed launches each, outside the tracer) and keeps the
// fastest for the key.  Tile variants give bit-identical results, so the choice never changes
// a number, only the time.
struct GemmTuner {
    struct Entry {
        int variant = 0;
        float us[GEMM_VARIANTS] = {};   // timed launch per variant (0: not valid for the shape)
    };
    bool enabled = true;
    int force = -1;   // >= 0: use this variant wherever it is valid (tests), no timing
    std::map<std::string, Entry> table;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~GemmTuner();
};
extern const char *const kGemmVariantNames[GEMM_VARIANTS];

// Dense FP64 MFMA GEMM C = A B (row-major, M%64 == K%16 == 0, N masked).
// kpad >= K: A's columns and B's rows exist (zero beyond K) up to kpad, so
// split-K ranges may run past K into them.  scratch (may be NULL) holds split-K
// partial products when the tile count is low.
void launch_dgemm(Tracer *t, hipStream_t s, const char *name, int M, int N, int K, int kpad,
                  const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                  double flops, double bytes, double *scratch, size_t scratch_doubles,
                  GemmTuner *tu = nullptr);
// (b2)+(c) at = Xvt Tt with the Lorentzian factor of column (E, j) and row F applied.
void launch_dgemm_lorentz(Tracer *t, hipStream_t s, int M, int N, int K, int kpad,
                          const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                          const double *Dlt, int nv_pad, const double *omega, double eps,
                          double occ, int ncp, double flops, double bytes, double *scratch,
                          size_t scratch_doubles, GemmTuner *tu = nullptr);
// Low-precision operator: FP32 gathered transforms, FP32 or split-BF16x3 dense transforms.
void launch_occ_transform_f32(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms,
                              const float *Xo, int no_pad, const double *dV, float *Tt,
                              int nc, const WorkSizes &ws);
void launch_occ_back_f32(Tracer *t, hipStream_t s, const BlockMapDev &bm, int n_atoms, int max_rows,
                         const float *Xo, int no_pad, int no_sum, const float *Ut, double *W, int nc,
                         const WorkSizes &ws);
void launch_sgemm(Tracer *t, hipStream_t s, const char *name, int M, int N, int K,
                  const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                  double flops, double bytes, const LorentzArgs *la, void *scratch,
                  size_t scratch_bytes, GemmTuner *tu = nullptr);
// Bhi/Blo: workspace of K * N uint16 each, filled with B's split (k-blocks of 8).
void launch_bgemm3(Tracer *t, hipStream_t s, const char *name, int M, int N, int K,
                   const uint16_t *Ahi, const uint16_t *Alo, int lda, const float *B, int ldb,
                   uint16_t *Bhi, uint16_t *Blo, float *C, int ldc, double flops, double bytes,
                   const LorentzArgs *la, void *scratch, size_t scratch_bytes);
void launch_to_f32(hipStream_t s, const double *x, float *y, int64_t n);
void launch_split_bf16(hipStream_t s, const double *x, uint16_t *hi, uint16_t *lo, int64_t n);

// (e) skinny K z for a few columns (HBM-streaming GEMV).
void launch_kmatvec_skinny(Tracer *t, hipStream_t s, int P_pad, const double *K,
                           const double *Zin, double *Zout, int nc, double P);

// ------------------------------------------------------------- Krylov support
struct Job {
    int32_t slot;
    int32_t type;     // JOB_RHS, JOB_ARNOLDI, JOB_RESID
    int32_t j;        // Arnoldi index (JOB_ARNOLDI); 1 = keep the warm-start x (JOB_RHS);
                      // cycle length (update_x); point index (alpha, store_x)
    int32_t drive;    // drive index of the slot's point
};
enum { JOB_RHS = 0, JOB_ARNOLDI = 1, JOB_RESID = 2 };

struct SlotsDev {
    double *V;        // [n_slots][m+1][P_pad] complex (interleaved)
    double *H;        // [n_slots][m(m+3)/2] complex, column j packed at j(j+3)/2, j+2 entries
    double *cs;       // [n_slots][m] real
    double *sn;       // [n_slots][m] complex
    double *g;        // [n_slots][m+1] complex
    double *x;        // [n_slots][P_pad] complex
    double *b;        // [n_slots][P_pad] complex
    double *hbuf;     // [n_slots][hbstride] scratch for Gram-Schmidt coefficients (>= 3m+4 complex)
    double *y;        // [n_slots][m] complex least-squares solution
    double *w;        // [n_slots][P_pad] complex: d + K x of the last true residual (d after b)
    int64_t vstride;  // doubles between slots in V  = (m+1)*P_pad*2
    int64_t hstride;  // doubles between slots in H
    int64_t hbstride; // doubles between slots in hbuf
    int m;
    int P_pad;
};

struct StepStatus {
    double value;     // JOB_RHS: ||b||; JOB_ARNOLDI: |g_{j+1}|; JOB_RESID: ||r||
    double hnext;     // JOB_ARNOLDI: h_{j+1,j}
    double eps_x;     // JOB_ARNOLDI with the error estimates on: eps_X and eps_P of Sec. 4.1
    double eps_p;
};

// Error estimates of the stopping test of Sec. 4.1 (DCGS2 steps only):
//   eps_X = ||A^-1|| ||r|| / ||X||,  eps_P = ||A^-1|| |d . r| / |P|,
// with ||A^-1|| taken as the Frobenius norm of R^-1, R the triangular factor
// of the cycle's Hessenberg matrix (the Krylov representation of A^-1 in the
// least-squares sense).  Kept incrementally: column k of Z = R^-1 from the
// column k of R, y = R^-1 g one column at a time, d.v_i and x0^H v_i per basis
// vector, and d.r = g_k phi_k with phi_k = -s_{k-1} phi_{k-1} + c_{k-1} d.v_k.
struct EpsDev {
    double *Z;          // [n_slots][zstride] complex: R^-1 by columns, column k at k(k+1)/2
    double *yv;         // [n_slots][m] complex: y = R^-1 g
    double *dl;         // [n_slots][m+1] complex: delta_i = d . v_i
    double *xi;         // [n_slots][m+1] complex: xi_i = x0^H v_i (x0 = the cycle's start)
    double *st;         // [n_slots][EPS_NS]: |Z|_F^2, P (2), S = x0^H V y (2), |y|^2, phi (2), |x0|^2
    const double *drives;   // [n_drive][P_pad] real
    int64_t zstride;    // doubles per slot in Z
};
constexpr int EPS_NS = 10;

void launch_gather_jobs(Tracer *t, hipStream_t s, const Job *jobs, int nb, const SlotsDev &sl,
                        double *Vb, int ncp, int P);
void launch_put_drive(Tracer *t, hipStream_t s, const Job *jobs, int nb, const double *drives,
                      int P_pad, double *Zin, int ncp, int P);
// Y = chi0 Zin; Zin = K x (residual jobs) or d (b jobs); drives [n_drive][P_pad].
void launch_post_jobs(Tracer *t, hipStream_t s, const Job *jobs, int nb, const SlotsDev &sl,
                      const double *Y, const double *Zin, const double *drives, int ncp, int P,
                      StepStatus *status);
void launch_arnoldi(Tracer *t, hipStream_t s, const Job *jobs, int nb, int jmax,
                    const SlotsDev &sl, int P, StepStatus *status, int n_arnoldi, double sum_j1);
// Arnoldi step with delayed reorthogonalisation (two passes over the basis).
// scratch (may be NULL) holds the partial sums of the split update (few jobs).
// eps (may be NULL) adds the error estimates of the stopping test to each step's status.
void launch_dcgs(Tracer *t, hipStream_t s, const Job *jobs, int nb, int jmax, const SlotsDev &sl, int P,
                 StepStatus *status, int n_arnoldi, double sum_j1, double *scratch = nullptr,
                 size_t scratch_doubles = 0, const EpsDev *eps = nullptr);
void launch_update_x(Tracer *t, hipStream_t s, const Job *jobs, int n, int jmax,
                     const SlotsDev &sl, int P, double sum_L);
// alpha[p][k] = -d_k . x of each finished point p (jobs[q].j); with `correct`
// the first-order term -(d_i + K x) . r of the point's own drive i is added
// to alpha[p][i] (r = the last true residual).  Rst, Wst (NULL, or
// [npts][P] complex) receive r and d_i + K x for the cross-drive terms.
void launch_alpha(Tracer *t, hipStream_t s, const Job *jobs, int n, const SlotsDev &sl,
                  const double *drives, int n_drive, int P_pad, int P, bool correct,
                  double *Rst, double *Wst, double *alpha_out);
// alpha[(w, i)][k] -= Wst[(w, k)] . Rst[(w, i)] for k != i (every frequency w).
void launch_alpha_cross(Tracer *t, hipStream_t s, int n_omega, int n_drive, int P, const double *Rst,
                        const double *Wst, double *alpha_out);
// learned warm start (kernels_mlp.hip)
void launch_mlp_gemm(hipStream_t s, int M, int N, int K, const float *A, int sam, int sak,
                     const float *B, int sbk, int sbn, float *C, int ldc);
void launch_features(hipStream_t s, int n, int n_pad, const double *omega, int nf, double scale,
                     float *phi);
void launch_bias_act(hipStream_t s, int M, int N, float *Z, const float *bias, int act);
void launch_mse(hipStream_t s, int M, int N, int n_rows, int n_cols, const float *out, const float *tgt,
                float *dout, float *loss);
void launch_tanh_back(hipStream_t s, int64_t n, const float *H, float *dH);
void launch_colsum(hipStream_t s, int M, int N, const float *dZ, float *db);
void launch_adam(hipStream_t s, int64_t n, float *p, const float *g, float *m, float *v, float lr,
                 float b1, float b2, float eps, int t);
void launch_gram(hipStream_t s, int n, const double *S, int64_t stride, int P, double *G);
void launch_basis(hipStream_t s, int n, int r, const double *S, int64_t stride, int P, const double *Wc,
                  double *U);
void launch_ws_apply(hipStream_t s, const Job *jobs, int n, const float *out, int ldo, const float *mean,
                     const float *sdev, int r, const double *U, int64_t ustride, double *x,
                     int64_t xstride, int P);
void launch_reset_slots(hipStream_t s, const Job *jobs, int n, const SlotsDev &sl, int P);
void launch_store_x(hipStream_t s, const Job *jobs, int n, const SlotsDev &sl, int P, double *out);

// ------------------------------------------------------ Lanczos (transition space)
constexpr int LZ_BLOCKS = 1024;   // most workgroups of the recursion's vector kernels
constexpr int LZ_GROUPS = 16;     // most vector groups of the reorthogonalisation update
// One block of nc <= 4 Lanczos recursions on Om2 = D^2 + S V_t^T f V_t S.
// The recursion's vectors are compact, tc x nc: transition (F, E) in row
// F * No + E (tc = No * Nv rounded up to 64, tail rows zero); the operator's
// buffer `at` keeps its layout, tp = Nv_pad * No_pad rows, row F * No_pad + E.
struct LanczosDev {
    double *R;             // basis: a ring of 3 vectors (ring = 1) or kmax + 1 vectors
    int64_t n;             // doubles per vector, tc * nc
    int64_t tc;            // compact rows
    int64_t tp;            // rows of `at`
    int64_t t_alg;         // transitions, No * Nv (also the tracer's work counts)
    int no, nv, no_pad;
    int ring, nc, kmax;
    int passes;            // Gram-Schmidt passes against the whole basis (0 with the ring)
    const double *St;      // [tc] sqrt(2 n D), 0 on the tail
    const double *D2t;     // [tc] D^2, 0 on the tail
    double *at;            // operator buffer: St q before the back half, V_t^T f V_t S q after the front half
    double *a, *b;         // [kmax][nc] recursion coefficients
    double *cn2;           // [nc] |c|^2
    int *len;              // [nc] recursion length (kmax until an invariant subspace ends it)
    int *step;             // current step (device counter)
    double *part;          // [LZ_BLOCKS][nc] partial sums
    // partial reorthogonalisation (null otherwise): Simon's estimates of q_j . q_i in a
    // ring of three rows [3][nc][kmax + 2], the running |T| estimate [nc], and the step's
    // decision: flag[0] = run the pass, flag[1] = the next step must run it too
    double *omega;
    double *anorm;
    int *flag;
};
void launch_lz_tables(hipStream_t s, const double *Dlt, int No, int Nv, int nv_pad, int64_t tc, double occ,
                      double *St, double *D2t);
// after the front half of the operator applied to the drives: q_0 = c / |c|, at = St q_0
void launch_lz_start(Tracer *t, hipStream_t s, const LanczosDev &L);
// after an operator pass on at = St q_j: a_j, b_j, q_{j+1} and at = St q_{j+1};
// without the ring, w is reorthogonalised against q_0..q_j (L.passes passes; j from the
// host, part2 [64 * (kmax + 1) * nc], h [(kmax + 1) * nc], part3 [LZ_GROUPS * tc * nc]).
void launch_lz_step(Tracer *t, hipStream_t s, const LanczosDev &L, int j, double *part2, double *h,
                    double *part3);
// Partial reorthogonalisation (L.omega, L.anorm, L.flag set): the head of step j
// ends with a_j, the norm b_j of the three-term residual and the device-side
// decision on the pass (L.flag[0]).  The whole step launches the gated pass and
// the second b_j every step (they return at once where the flag is clear); no
// host synchronisation.  The tail runs npass passes against q_0..q_j (then b_j
// again) and the normalisation, for a caller that has read the flag.
void launch_lz_step_head(Tracer *t, hipStream_t s, const LanczosDev &L, int j);
void launch_lz_step_partial(Tracer *t, hipStream_t s, const LanczosDev &L, int j, double *part2, double *h,
                            double *part3);
void launch_lz_step_tail(Tracer *t, hipStream_t s, const LanczosDev &L, int j, int npass, double *part2, double *h,
                         double *part3);
// Solutions of eq. sle from the stored basis, LZ_XCOL / nc frequencies per pass
// (omega [LZ_XCOL / nc], nw of them valid): y = |c| (T_k - z)^-1 e_1 (dw
// [kuse][LZ_XCOL][4], Y [kuse][LZ_XCOL] complex), then at = St Q_k y in the
// operator's layout with 2 (LZ_XCOL / nc) nc real columns, for the back half.
constexpr int LZ_XCOL = 16;
void launch_lz_solution_cols(Tracer *t, hipStream_t s, const LanczosDev &L, int kuse, const int *len,
                             const double *omega, int nw, double eps, double *dw, double *Y, double *at);
// From Yb = B Q_k y [P_pad][2M]: x rows [nw][nc][P] complex (= -Yb) and alpha [nw][nc][nc]
// complex (alpha_ki = -d_k . x_i; drives [nc][P]); either output may be NULL.
void launch_lz_solution_out(hipStream_t s, const double *Yb, int nc, int nw, int P, const double *drives,
                            double *x_rows, double *alpha);
// alpha(omega) [n_omega][nc] complex from the first min(kuse, len[s]) coefficients
void launch_lz_cfrac(hipStream_t s, const double *a, const double *b, int nc, int kuse, const int *len,
                     const double *cn2, const double *omega, int n_omega, double eps, double *out);

// two-sided Lanczos (chi0_solve_bilanczos): per-point vector work of the recursion
void launch_bl_drives(hipStream_t s, int P, int P_pad, int np, int p0, int n_drive, const double *D, double *Zin);
void launch_bl_init(hipStream_t s, int P, int npts, int p0, int n_drive, const double *D, int P_pad,
                    const double *Yb, int ldb, double *V1, double *W1, double *V0, double *W0, int ld,
                    double *beta, int ldbeta, double *bnorm, int *flag);
void launch_bl_pack(hipStream_t s, int P_pad, int nc, const double *KV, const double *W1, double *Zin);
void launch_bl_unpack(hipStream_t s, int P, int P_pad, int nc, const double *Yout, double *CW);
void launch_bl_step(hipStream_t s, int npts, int P, int k, const double *Yout, const double *KCW,
                    const double *V1, const double *W1, double *V0, double *W0, int ld, double *alpha,
                    int ldalpha, double *beta, int ldbeta, double *rnorm, int ldrn, int *flag);

// apply: caller rows [r][P] complex <-> operator columns [P_pad][ncp]
void launch_rows_to_cols(Tracer *t, hipStream_t s, const double *z, int nb, int P,
                         double *Zin, int ncp);
void launch_cols_to_rows(Tracer *t, hipStream_t s, const double *Y, int nb, int P, int ncp,
                         double *out);
void launch_zero(Tracer *t, hipStream_t s, double *p, int64_t n);

}  // namespace chi0
