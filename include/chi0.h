/*
 * chi0.h -- C-ABI of the MI355X (gfx950) iterative polarizability library.
 *
 * The library computes the interacting dynamical polarizability of a
 * molecule described in a basis of dominant products, following
 * P. Koval, D. Foerster, O. Coulaud, "A Parallel Iterative Method for
 * Computing Molecular Absorption Spectra" (2010):
 *
 *   chi0_{mu nu}(w) = sum_{E occ, F virt} v_mu^{EF} L_EF(w) v_nu^{EF},
 *       v_mu^{EF} = X_a^E V_mu^{ab} X_b^F                     (Sec. 3, eq. response-mat)
 *       L_EF(w)   = n [1/(w - D_EF + i eps) - 1/(w + D_EF + i eps)],  D_EF = e_F - e_E
 *   (1 - chi0(w) K) x(w) = chi0(w) d                           (Sec. 4.1, eq. sle)
 *   alpha_{ki}(w) = -d_k . x_i(w)       (eq. eqpolarizability; sign: alpha = -P)
 *
 * chi0 is never formed: chi0(w) z is applied matrix-free by the factored
 * sequence of Sec. 4.2 (Table t:flops): vertex contraction, the occupied and
 * virtual orbital transforms, the frequency factor, and the contraction back
 * onto products.  The linear system is solved by GMRES (Sec. 4.1).
 *
 * Conventions
 *   - Units: Hartree and Bohr.  Energies must already be shifted so that the
 *     n_occ occupied eigenvalues are < 0 and the virtual ones > 0 (Sec. 2).
 *   - Complex numbers are interleaved (re, im) pairs of double, i.e. the
 *     layout of C99 `double _Complex` / std::complex<double> / torch.complex128.
 *   - Matrices are row-major.
 *   - Return codes: 0 success, > 0 warning, < 0 error.  No exception or
 *     abort crosses the ABI; chi0_last_error() gives a message.
 *   - A context is not thread-safe: use one context per host thread.  Calls
 *     that take a hipStream_t enqueue work on that stream and return without
 *     synchronising it; every other call is synchronous.
 */
#ifndef CHI0_H
#define CHI0_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define CHI0_OK               0
#define CHI0_NOT_CONVERGED    1   /* warning: some points missed the tolerance; results still written */
#define CHI0_EINVAL          (-1) /* bad size, pointer, index or parameter */
#define CHI0_ENOSYS          (-2) /* no system set on this context (or host-only context) */
#define CHI0_ENOMEM          (-3) /* device or host allocation failed */
#define CHI0_EHIP            (-4) /* a HIP runtime call failed; message names it */
#define CHI0_ENONFINITE      (-5) /* NaN or Inf in an input */
#define CHI0_EASYM           (-6) /* vertex block or kernel matrix not symmetric */

/* Arithmetic of the orbital transforms inside chi0 (Table t:flops steps 2-5).
 * The vertex contractions, the frequency factor, K, Gram-Schmidt, the
 * Hessenberg problem and the true residual are always FP64.
 *   FP64    every transform on FP64 matrix cores.
 *   FP32    transforms on FP32 matrix cores, FP32 intermediates.
 *   BF16X3  the two dense virtual-orbital transforms as split BF16 x 3 (each
 *           operand x = bf16 hi + bf16 lo, three BF16 products, FP32
 *           accumulation); the block-sparse occupied transforms in FP32. */
#define CHI0_PREC_FP64        0
#define CHI0_PREC_FP32        1
#define CHI0_PREC_BF16X3      2

typedef struct chi0_ctx chi0_ctx;      /* opaque */

/*
 * Create a context bound to HIP device `device` (an index as for
 * hipSetDevice).  device = -1 creates a host-only context: chi0_set_system
 * then validates its inputs and builds the host-side block maps but uploads
 * nothing; calls that compute return CHI0_ENOSYS.  *out is NULL on failure.
 */
int chi0_create(chi0_ctx **out, int device);

/* Release every device and host resource of the context (NULL is a no-op). */
void chi0_destroy(chi0_ctx *ctx);

/* Message of the last failing call on this context ("" if none).  The
 * pointer stays valid until the next call on the same context.  ctx may be
 * NULL, then the message of the last failed chi0_create is returned. */
const char *chi0_last_error(const chi0_ctx *ctx);

/*
 * Define the molecule (Sec. 2-3).  All pointers are host memory, read during
 * the call and not retained; the context keeps its own device copies.  A
 * later call replaces the system.
 *
 *  n_atoms, positions   number of atoms; positions [n_atoms][3] in Bohr (may
 *                       be NULL; only checked for finiteness).
 *  n_orb, n_occ         atomic orbitals N (= molecular orbitals) and occupied
 *                       states, 1 <= n_occ < n_orb.
 *  occ_factor           occupation n of an occupied state (2 for a closed
 *                       shell); virtual states carry 0.
 *  eigenvalues          [n_orb] Kohn-Sham energies, the first n_occ < 0 and
 *                       the rest > 0.
 *  X                    [n_orb][n_orb], X[a*n_orb + E] = X_a^E, coefficient of
 *                       atomic orbital a in molecular orbital E (eq. lcao).
 *  atom_orb_offset      [n_atoms+1] atomic orbitals of atom A are
 *                       [offset[A], offset[A+1]); offset[0] = 0,
 *                       offset[n_atoms] = n_orb, strictly increasing.
 *  n_prod, prod_atoms   number of dominant products; prod_atoms[2*mu] = atom
 *                       A of product mu, prod_atoms[2*mu+1] = atom B != A of
 *                       a bilocal product or -1 for a local one (Sec. 3).
 *  vblock_offset        [n_prod+1] start of each product's vertex block in
 *                       `vblock`; vblock_offset[0] = 0 and consecutive
 *                       differences equal s_mu^2.
 *  vblock               the vertex V_mu^{ab} of each product as a dense
 *                       symmetric s_mu x s_mu row-major block over its support:
 *                       the orbitals of A, then (bilocal) those of B; s_mu is
 *                       the number of those orbitals (eq. vertex-ansatz).
 *  K                    [n_prod][n_prod] symmetric interaction kernel f_Hxc
 *                       (Sec. 5), frequency independent.
 *
 * Errors: CHI0_EINVAL (sizes, offsets, indices, energies not shifted,
 * occ_factor <= 0), CHI0_ENONFINITE, CHI0_EASYM (a block or K asymmetric by
 * more than 1e-12 of its largest entry), CHI0_ENOMEM, CHI0_EHIP.  On error
 * the previous system is gone and the context has none.
 */
int chi0_set_system(chi0_ctx *ctx,
                    int32_t n_atoms, const double *positions,
                    int32_t n_orb, int32_t n_occ, double occ_factor,
                    const double *eigenvalues, const double *X,
                    const int32_t *atom_orb_offset,
                    int32_t n_prod, const int32_t *prod_atoms,
                    const int64_t *vblock_offset, const double *vblock,
                    const double *K);

/* Sizes of the current system: any pointer may be NULL.  CHI0_ENOSYS if none. */
int chi0_get_sizes(const chi0_ctx *ctx, int32_t *n_orb, int32_t *n_occ,
                   int32_t *n_prod, int32_t *n_atoms);

/*
 * out_r = chi0(omega[r]) z_r for r < n_rhs (Sec. 4.2, matrix-free).
 *
 *  omega   host [n_rhs] frequencies (Ha), any real values.
 *  eps     broadening (Ha), > 0.
 *  z, out  DEVICE buffers of n_rhs * n_prod complex values (interleaved
 *          doubles), row r at offset r*n_prod.  Owned by the caller; may not
 *          overlap.  Work is enqueued on `stream` (a hipStream_t, NULL = the
 *          default stream) and the call returns before it completes.  The
 *          context's workspace is shared by all calls on the context, so do
 *          not overlap two calls on one context on different streams.
 *  precision  CHI0_PREC_FP64, CHI0_PREC_FP32 or CHI0_PREC_BF16X3.
 */
int chi0_apply(chi0_ctx *ctx, int32_t n_rhs, const double *omega, double eps,
               const double *z, double *out, int32_t precision, void *stream);

/*
 * chi0_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same FP64 operator (precision is always CHI0_PREC_FP64), with every
 * workspace buffer taken from a static device array of
 * CHI0_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its first
 * chi0_create on that GPU until the process ends; the call itself allocates
 * nothing (no hipMalloc, no events, no tile tuning).  Results equal
 * chi0_apply's up to rounding (the GEMMs' split-K partial sums may differ).
 *
 *  omega, eps, z, out, stream   as for chi0_apply (z, out DEVICE buffers).
 * The array is shared by every context and call on the GPU and keeps the last
 * call's contents (each call clears what it needs): calls that overlap on one
 * GPU (two streams, two threads) race and must be serialised by the caller.
 * Errors: as chi0_apply, and CHI0_EINVAL when n_rhs needs more workspace than
 * the array holds (the message says how many right-hand sides fit: 16
 * for 540 orbitals and 3.3k products, 1 for 1800 orbitals and 12k products).
 */
#define CHI0_NOALLOC_SCRATCH_BYTES (128LL << 20)
int chi0_apply_noalloc(chi0_ctx *ctx, int32_t n_rhs, const double *omega, double eps,
                       const double *z, double *out, void *stream);

/*
 * Replay chi0_apply from a HIP graph (enable != 0; default off).  A call with
 * n_rhs <= 256 is captured the second time its (n_rhs, precision, z, out,
 * eps) repeat (the first such call runs eagerly and tunes the GEMM tiles) and
 * replayed while they keep repeating: the frequencies are copied to the
 * device before each replay, the vectors z are read at replay time.  For
 * callers that apply chi0 many times to the same buffers, e.g. their own
 * Krylov loop on a small system, where launching the ~10 kernels of a pass
 * costs as much as running them.  The graph is dropped when the system or the
 * workspaces change, while kernel timing (chi0_set_timing) is on no graph is
 * used.  Synchronises the device.
 */
int chi0_set_graphs(chi0_ctx *ctx, int32_t enable);

/* Options of chi0_solve_response.  Zero-initialise, then set what you need;
 * chi0_solve_opts_default() fills the defaults. */
typedef struct chi0_ws chi0_ws;        /* learned warm start (see chi0_ws_fit) */

typedef struct chi0_solve_opts {
    int32_t restart;      /* GMRES(m) Krylov dimension per cycle, 1..32767 (4095 with CGS2;
                             default 30); the basis needs (m+2) n_prod 16 bytes per slot */
    int32_t max_iter;     /* cap on Arnoldi steps per point (default 10000) */
    double  tol;          /* stop when ||chi0 d - A x||_2 <= tol ||chi0 d||_2 (default 1e-10) */
    int32_t precision;    /* CHI0_PREC_* of the Arnoldi steps (default FP64); b = chi0 d and
                             every true residual are FP64 (iterative refinement) */
    int32_t batch;        /* (omega, drive) points solved concurrently, 1..256; 1 = one at a time.
                             Capped at what fits in free device memory: each point holds
                             (restart+2) n_prod 16 + restart^2 8 bytes of Krylov basis and
                             Hessenberg matrix (twice the latter with the eps stopping tests) */
    double  inner_tol;    /* low precision only: a cycle ends when the Arnoldi residual
                             estimate falls by this factor (0 = 1e-6 for FP32, 1e-4 for BF16X3) */
    const chi0_ws *warm;  /* NULL, or a warm start fitted on this context and system: every point
                             starts from x0 = U c(omega) instead of 0, unless
                             ||chi0 d - A x0|| >= ||chi0 d||, then from 0 */
    int32_t ortho;        /* CHI0_ORTHO_*: Gram-Schmidt variant of the Arnoldi step */
    int32_t lanes;        /* 0 = auto (2 when batch >= 16, else 1), or 1..4: the concurrent
                             slots are dealt to this many lanes, each with its own stream and
                             operator workspace, so that one lane's memory-bound Gram-Schmidt
                             passes overlap the other's matrix-core transforms */
    int32_t stop;         /* CHI0_STOP_*: the test that ends a point (default: residual) */
    int32_t alpha_form;   /* CHI0_ALPHA_*: how alpha is formed from the final iterate
                             (default CHI0_ALPHA_CORRECTED) */
    const double *x0;     /* NULL, or DEVICE memory [n_omega][n_drive][n_prod] complex: point
                             (omega_i, drive k) starts from x0[i][k] instead of 0 (for example the
                             solution at a neighbouring frequency), unless
                             ||chi0 d - A x0|| >= ||chi0 d||, then from 0; not with `warm` */
    const chi0_ws *const *warm_drive;   /* NULL, or host [n_drive]: a learned warm start for each
                             drive (an entry may be NULL: that drive starts from 0), each fitted on
                             this context and system, typically on its own drive's solutions; not
                             with `warm` or `x0` */
    int32_t mixed;        /* precision != FP64 only: CHI0_MIXED_REFINE (default) or _RELAXED */
    double  relax;        /* CHI0_MIXED_RELAXED: switch to `precision` once the residual estimate is
                             at most relax tol ||chi0 d|| / u, u the low-precision operator's
                             relative error (3e-7 FP32, 6e-6 BF16X3); 0 = 1 */
} chi0_solve_opts;

/* How a low-precision operator enters the solve (precision != FP64).  Both end
 * every cycle with an FP64 true residual, so the stopping test is unchanged.
 *   REFINE   iterative refinement: each cycle runs all its Arnoldi steps in
 *            low precision and ends when its residual estimate has fallen by
 *            inner_tol (or met tol); the FP64 residual then starts the next.
 *   RELAXED  one Krylov space as in FP64, whose operator precision is relaxed
 *            as the residual falls (inexact Krylov: a step may apply an
 *            operator with relative error up to ~tol ||b|| / ||r_k||): FP64
 *            steps until the estimate reaches relax tol ||b|| / u, then
 *            low-precision steps; the cycle ends on the estimate at tol.
 * In both, a low-precision cycle whose true residual did not halve hands the
 * point to FP64 steps (stats.fallback). */
#define CHI0_MIXED_REFINE     0
#define CHI0_MIXED_RELAXED    1

/* Stopping test of a point (Sec. 4.1).
 *   RESIDUAL  the true relative residual ||chi0 d - A x|| / ||chi0 d|| <= tol
 *             (confirmed by an FP64 residual at the end of each cycle).
 *   EPS_P     the paper's estimate of the relative error of the polarizability,
 *             eps_P = ||A^-1|| |d . r| / |d . x| <= tol, where ||A^-1|| is the
 *             Frobenius norm of the inverse triangular factor of the cycle's
 *             Hessenberg matrix (the Krylov representation of A^-1) and r the
 *             GMRES residual; the paper's choice for percent-level tolerances.
 *   EPS_PX    the paper's combined test: eps_P <= tol and
 *             eps_X = ||A^-1|| ||r|| / ||x|| <= tol.
 * The estimates need DCGS2 steps and FP64 precision, and R^-1 of each slot's
 * cycle: restart (restart + 1) 8 extra bytes per concurrent point.  A point
 * whose cycle ends by the estimate counts as converged; its stats carry the
 * estimates and the true residual of the solution returned. */
#define CHI0_STOP_RESIDUAL    0
#define CHI0_STOP_EPS_P       1
#define CHI0_STOP_EPS_PX      2

/* Polarizability from the final iterate x_i of drive i and its FP64 true
 * residual r_i = chi0 d_i - A x_i (Sec. 4.1 gives the error of P = d . x as
 * d . A^-1 r).
 *   CORRECTED  alpha_ki = -(d_k . x_i + (d_k + K x_k) . r_i): d_k + K x_k is
 *              A^-T d_k at the exact x_k (chi0 and K are complex symmetric, so
 *              A^T = 1 - K chi0), so the residual term is taken to first order
 *              and the error of alpha is second order in the residuals, where
 *              -d_k . x_i alone is first order.  K x_k and r_i come from the
 *              last true-residual computation of each point at no extra
 *              operator cost.  With more than one drive the call keeps r and
 *              d + K x of every point on the device for the cross terms:
 *              n_omega n_drive n_prod 32 extra bytes for the call.
 *   PLAIN      alpha_ki = -d_k . x_i (eq. eqpolarizability as written). */
#define CHI0_ALPHA_CORRECTED  0
#define CHI0_ALPHA_PLAIN      1

/* Gram-Schmidt of the Arnoldi step (eq. orthogonal-krylov-basis, done twice).
 *   CGS2   two classical passes per step: four reads of the basis.
 *   DCGS2  the second pass of each vector is delayed into the next step and
 *          fused with its projection: two reads of the basis per step; the
 *          newest column is provisional until the next step, so the basis
 *          holds one extra vector (m+2 per point) and the residual estimate
 *          lags one step.
 *   AUTO   DCGS2 when restart >= 8, else CGS2. */
#define CHI0_ORTHO_AUTO       0
#define CHI0_ORTHO_CGS2       1
#define CHI0_ORTHO_DCGS2      2

/* Per-point solver record (one per omega and drive). */
typedef struct chi0_point_stats {
    int32_t iterations;   /* Arnoldi steps (operator applications, excluding b and residual checks) */
    int32_t restarts;     /* completed GMRES cycles (each ends with an FP64 true residual) */
    int32_t converged;    /* 1 if the true relative residual met tol */
    int32_t breakdown;    /* 1 if the Krylov space became invariant (exact solution) */
    int32_t fallback;     /* 1 if a low-precision point switched to FP64 steps after a cycle
                             that did not halve the true residual */
    int32_t warm_start;   /* 0 none, 1 started from the warm start, 2 warm start rejected */
    double  rel_residual; /* true ||b - A x|| / ||b|| at exit */
    double  warm_rel0;    /* ||b - A x0|| / ||b|| of the warm start (0 if none) */
    double  eps_x;        /* CHI0_STOP_EPS_*: the last eps_X and eps_P estimates seen (else 0) */
    double  eps_p;
    int32_t low_prec_steps; /* of `iterations`, the Arnoldi steps that applied chi0 with the
                               reduced-precision transforms (0 for CHI0_PREC_FP64) */
    int32_t reserved;
} chi0_point_stats;

void chi0_solve_opts_default(chi0_solve_opts *opts);

/*
 * Polarizability tensor over a frequency grid (Sec. 4.1 and Algorithm a:main):
 * for each omega[w] and each drive i, GMRES solves (1 - chi0 K) x = chi0 d_i
 * from x = 0, then alpha[w][k][i] = -d_k . x for every drive k, with the
 * residual term of CHI0_ALPHA_CORRECTED unless opts->alpha_form says PLAIN.
 *
 *  omega    host [n_omega] (Ha).
 *  eps      broadening (Ha), > 0.
 *  n_drive  1..3 drives; V_ext host [n_drive][n_prod] real dipole vectors.
 *  opts     NULL for the defaults.
 *  alpha    host [n_omega][n_drive][n_drive] complex (interleaved), written.
 *  stats    host [n_omega][n_drive] records, may be NULL.
 * Returns CHI0_OK, CHI0_NOT_CONVERGED (alpha from the last iterate), or an
 * error.  Synchronous; uses the context's own stream.
 */
int chi0_solve_response(chi0_ctx *ctx, int32_t n_omega, const double *omega, double eps,
                        int32_t n_drive, const double *V_ext,
                        const chi0_solve_opts *opts,
                        double *alpha, chi0_point_stats *stats);

/*
 * chi0_solve_response that also returns the solutions: the induced density
 * response x = delta n(omega) of eq. sle in the product basis, for every
 * point.
 *
 *  x   host [n_omega][n_drive][n_prod] complex (interleaved doubles), written;
 *      x[w][i] solves (1 - chi0(omega[w]) K) x = chi0(omega[w]) d_i.
 * The call needs n_omega * n_drive * n_prod * 16 bytes of extra device
 * memory for the duration of the call.  Everything else as chi0_solve_response.
 */
int chi0_solve_response_x(chi0_ctx *ctx, int32_t n_omega, const double *omega, double eps,
                          int32_t n_drive, const double *V_ext, const chi0_solve_opts *opts,
                          double *alpha, chi0_point_stats *stats, double *x);

/*
 * Learned warm start.  The paper starts GMRES from 0 (Sec. 4.1); this adds an
 * initial guess learned from solutions at training frequencies:
 *   1. plain FP64 GMRES solves (1 - chi0 K) x = chi0 d at the n_train
 *      frequencies omega_train (one drive d, host [n_prod]);
 *   2. U = the `rank` leading left singular vectors of the solutions (from
 *      the eigen-decomposition of their Gram matrix);
 *   3. a 3-layer perceptron (tanh, `width` units) maps the Fourier features
 *      sin/cos(k pi omega / w_scale), k = 1..n_freq, to the coordinates
 *      c = U^H x of the training solutions; it is trained by full-batch Adam
 *      with FP32 weights and BF16 matrix-core products;
 *   4. x0(omega) = U c(omega).
 * Everything runs on the context's device.  The warm start belongs to the
 * context and system it was fitted on and must be freed before the context.
 */
typedef struct chi0_ws_cfg {
    int32_t rank;         /* basis size r <= n_train (default 64) */
    int32_t width;        /* hidden units, multiple of 32 (default 256) */
    int32_t n_freq;       /* Fourier modes, 16 or 32 (default 16: 32 input features) */
    int32_t epochs;       /* Adam steps (default 3000) */
    double  w_scale;      /* feature period scale (0 = max |omega_train|) */
    double  lr;           /* Adam learning rate (default 2e-3, cosine decay to 1e-2 of it) */
    uint64_t seed;        /* weight initialisation */
    int32_t restart;      /* training solves: GMRES(m) (0 = n_prod) */
    int32_t batch;        /* training solves: concurrent points (default 64) */
    double  tol;          /* training solves: tolerance (default 1e-10) */
    int32_t reserved[4];  /* must be zero */
} chi0_ws_cfg;

void chi0_ws_cfg_default(chi0_ws_cfg *cfg);

/* Fit a warm start (see above).  *out is NULL on failure. */
int chi0_ws_fit(chi0_ctx *ctx, int32_t n_train, const double *omega_train, double eps,
                const double *drive, const chi0_ws_cfg *cfg, chi0_ws **out);

void chi0_ws_free(chi0_ws *ws);

/* x0[i] = U c(omega[i]) into DEVICE memory x0 [n][n_prod] complex; synchronous. */
int chi0_ws_predict(chi0_ws *ws, int32_t n, const double *omega, double *x0);

/* Training loss (mean squared error of the normalised coordinates) after
 * each Adam step; copies min(cap, epochs) values, returns epochs. */
int chi0_ws_loss_history(const chi0_ws *ws, float *loss, int32_t cap);

/*
 * Spectrum, poles and residues from a Lanczos recursion in transition space.
 *
 * On the T = n_occ * n_virt transitions (E occupied, F virtual) the
 * response has the pole form (Sec. 3 with eq. sle; Casida's equations):
 *   Om2 = diag(D^2) + S V_t^T K V_t S,  S = diag(sqrt(2 n D)),  c = S V_t^T d,
 *   alpha(w) = c^T (Om2 - (w + i eps)^2)^-1 c,
 * with D_EF = e_F - e_E and V_t the n_prod x T matrix of the transition
 * vertices v_mu^{EF}.  chi0_lanczos runs the symmetric Lanczos recursion
 *   q_0 = c / |c|,   b_j q_{j+1} = Om2 q_j - a_j q_j - b_{j-1} q_{j-1},
 * applying Om2 matrix-free with the chi0 operator's kernels, for up to four
 * drives at once.  The k x k tridiagonal T_k (diagonal a, off-diagonal b)
 * then gives, for every frequency at once,
 *   alpha_k(w) = |c|^2 e_1^T (T_k - (w + i eps)^2)^-1 e_1
 *             = sum_j r_j / (theta_j - (w + i eps)^2),
 * theta_j the eigenvalues of T_k (poles of alpha in (w + i eps)^2, i.e.
 * excitation energies sqrt(theta_j)) and r_j = |c|^2 (u_j)_1^2 their residues.
 * This is the economical treatment of the frequency axis, with pole
 * positions and strengths, that the paper names as further work (Sec. 8).
 * The continued fraction yields the diagonal alpha_ii of each drive; with a
 * stored basis (any reorthogonalised recursion) the solutions of eq. sle and
 * the full tensor alpha_ki follow at requested frequencies (n_x below).
 */
typedef struct chi0_lanczos_opts {
    int32_t k_max;        /* most steps (default 4000); capped to n_occ * n_virt */
    int32_t reorth;       /* CHI0_LZ_REORTH_PARTIAL (default), _FULL, _FULL2 or _NONE */
    double  tol;          /* > 0: stop once alpha_k at the check frequencies changes by at most tol
                             between two consecutive pairs of checks, the change of each point relative
                             to max(|Im alpha_k|, 1e-3 max over the check points of |Im alpha_k|);
                             0: run k_max steps (default) */
    int32_t check_every;  /* steps between checks (default 100) */
    int32_t n_check;      /* number of check frequencies (0: no checks) */
    const double *omega_check;   /* host [n_check], Ha */
    double  eps;          /* broadening of the checks, Ha (> 0 when n_check > 0) */
    int32_t graph;        /* 1: after the first step, replay each step's launch sequence from one
                             HIP graph (CHI0_LZ_REORTH_NONE, timing off); 0 (default): launch eagerly */
    int32_t n_x;          /* > 0: also the solutions of eq. sle at n_x frequencies (needs a stored
                             basis: any mode but CHI0_LZ_REORTH_NONE; and eps > 0) */
    const double *omega_x;   /* host [n_x], Ha */
    double *x;            /* host [n_x][n_drive][n_prod] complex, or NULL: x_i(w) = -B Q_k y(w),
                             B = V_t S, y = |c_i| (T_k - (w + i eps)^2)^-1 e_1, k = len[i]; with
                             CHI0_LZ_REORTH_PARTIAL (the default) the basis is orthogonal only to
                             about sqrt(machine epsilon) and x, alpha_x are good to ~1e-7 relative
                             (what the tests hold them to); use CHI0_LZ_REORTH_FULL, which keeps the
                             basis orthogonal to rounding, for solutions at the FP64 bar */
    double *alpha_x;      /* host [n_x][n_drive][n_drive] complex, or NULL: the full tensor
                             alpha_ki(w) = -d_k . x_i(w) (eq. eqpolarizability, alpha = -P) */
    int32_t reserved[2];  /* must be zero */
} chi0_lanczos_opts;

/* Three-term recurrence only: three transition vectors in device memory.  The
 * recursion loses orthogonality as soon as a Ritz value converges; its
 * spectrum then converges far more slowly (on spectra with outlying poles,
 * as the Coulomb-like kernels give, not within T steps). */
#define CHI0_LZ_REORTH_NONE   0
/* After the three-term step each new vector is orthogonalised against every
 * previous one by one classical Gram-Schmidt pass (FULL2: two passes): k_max
 * + 1 vectors in device memory (CHI0_ENOMEM if they do not fit).  One pass
 * keeps the basis orthogonal to rounding here, because the three-term step
 * leaves only small components along the old vectors. */
#define CHI0_LZ_REORTH_FULL   1
#define CHI0_LZ_REORTH_FULL2  2
/* Partial reorthogonalisation (Simon's omega recurrence, advanced on the device
 * from a_j and b_j): a step runs the pass only when the estimated loss of
 * orthogonality of the new vector exceeds sqrt(machine epsilon), and then the
 * next step too; the decision is a device flag, so the host is not waited on
 * between convergence checks.  Same memory as FULL. */
#define CHI0_LZ_REORTH_PARTIAL 3

void chi0_lanczos_opts_default(chi0_lanczos_opts *opts);

/* Run the recursion for n_drive (1..4) drives, host [n_drive][n_prod]
 * (NULL opts: defaults).  Writes to host memory, per drive s:
 * a[s * k_max + j], b[s * k_max + j] for j < len[s] (0 beyond), c_norm2[s]
 * = |c_s|^2 and len[s], the number of valid coefficients: the steps run, or
 * fewer where an invariant subspace ended the recursion (then T_len is
 * exact and b[len - 1] = 0); a drive with c = 0 has len 0 (alpha = 0).
 * b[len - 1] is otherwise the norm of the next Lanczos vector (T_len uses
 * b[0 .. len - 2]).  Synchronous, on the context's stream.  Returns CHI0_OK,
 * CHI0_NOT_CONVERGED when tol > 0 and k_max steps did not meet it (the
 * coefficients are still written), or an error: CHI0_EINVAL (sizes,
 * options), CHI0_ENONFINITE, CHI0_ENOSYS (no system), CHI0_ENOMEM. */
int chi0_lanczos(chi0_ctx *ctx, int32_t n_drive, const double *drives, const chi0_lanczos_opts *opts,
                 double *a, double *b, double *c_norm2, int32_t *len);

/* alpha_k(omega) of each drive, computed on the device as the continued
 * fraction of T_k: alpha [n_omega][n_drive] complex (host), from the first
 * len[s] coefficients of drive s in a, b (host, [n_drive][ld]) and
 * c_norm2[s].  Synchronous.  CHI0_EINVAL for len outside 0..ld or eps <= 0. */
int chi0_lanczos_spectrum(chi0_ctx *ctx, int32_t n_drive, int32_t ld, const double *a, const double *b,
                          const double *c_norm2, const int32_t *len, int32_t n_omega, const double *omega,
                          double eps, double *alpha);

/* Poles and residues of alpha_k for one drive: theta[0..k) the eigenvalues
 * of T_k (diagonal a[0..k), off-diagonal b[0..k-1)) in ascending order and
 * resid[j] = c_norm2 (u_j)_1^2.  A host computation on the k x k tridiagonal
 * matrix (implicit QR steps with Wilkinson shifts, O(k^2)); needs no
 * context.  CHI0_EINVAL (k < 1, NULL, c_norm2 < 0), CHI0_ENONFINITE, or
 * CHI0_NOT_CONVERGED if the QR iteration does not converge. */
int chi0_lanczos_poles(int32_t k, const double *a, const double *b, double c_norm2, double *theta,
                       double *resid);

/*
 * Polarizability by the two-sided (biorthogonal) Lanczos recursion on
 * A = 1 - chi0(w) K: the Krylov method that the Sec. 4 introduction says the
 * authors used before the solve of eq. sle, there to build a representation
 * of A that is easy to invert within its Krylov subspace.  One recursion per
 * (omega, drive) point, in the bilinear form x^T y: right start chi0 d, left
 * start d, T_k complex symmetric tridiagonal, and
 *     alpha_ii(w) = -beta_1^2 e_1^T T_k^-1 e_1     (beta_1^2 = d^T chi0 d).
 * Each step applies A and A^T = 1 - K chi0 (two K products and one chi0 pass
 * over two vectors per point) and keeps three vectors per side: no stored
 * basis and no reorthogonalisation.  A point stops when the residual
 * |chi0 d - A x_k| / |chi0 d| of x_k = V_k T_k^-1 beta_1 e_1 (evaluated for
 * every step from the recurrence; the host reads the coefficients back every
 * 10 steps, so a point may run up to 9 steps past its answer) is <= tol, at a
 * breakdown (s^T r exactly zero, or an invariant subspace: |r| <= 1e-13 |A v|;
 * there is no look-ahead), or after max_steps.  Up to 64 points run at once.
 *
 *  omega      host [n_omega] (Ha); eps > 0 (Ha).
 *  n_drive    1..3; drives host [n_drive][n_prod] real.
 *  tol        > 0; max_steps >= 1 (the coefficients of max_steps steps per
 *             point are held on the device: 40 bytes per step and point).
 *  alpha      host [n_omega][n_drive] complex (interleaved), alpha_ii of each
 *             point at its last step, written.
 *  steps      host [n_omega][n_drive] steps taken, may be NULL.
 *  status     host [n_omega][n_drive]: 0 converged, 1 max_steps reached,
 *             2 breakdown before tol; may be NULL.
 * Returns CHI0_OK, CHI0_NOT_CONVERGED (some point has status 1 or 2), or an
 * error (CHI0_EINVAL, CHI0_ENONFINITE, CHI0_ENOSYS, CHI0_ENOMEM, CHI0_EHIP).
 * Synchronous; uses the context's own stream.
 */
int chi0_solve_bilanczos(chi0_ctx *ctx, int32_t n_omega, const double *omega, double eps, int32_t n_drive,
                         const double *drives, double tol, int32_t max_steps, double *alpha, int32_t *steps,
                         int32_t *status);

/*
 * Kernel timing (tracing).  When enabled, every kernel launch of the
 * library is bracketed by HIP events on the stream it runs on, and the
 * durations are accumulated per kernel name, together with the algorithmic
 * work of each launch (unpadded sizes; every operand counted once).
 * chi0_kernel_stats copies up to `cap` records and returns how
 * many kernels have records.  Reading the records synchronises the
 * context's streams.  Disabled by default; enabling resets the records.
 */
typedef struct chi0_kernel_record {
    char    name[48];
    int64_t launches;
    double  total_ms;
    double  flops;        /* algorithmic floating-point operations of those launches */
    double  bytes;        /* algorithmic HBM bytes (each operand read or written once) */
} chi0_kernel_record;

int chi0_set_timing(chi0_ctx *ctx, int32_t enable);
int chi0_kernel_stats(chi0_ctx *ctx, chi0_kernel_record *records, int32_t cap);

/* Restrict timing to the kernels named in `names` (comma-separated record
 * names as reported by chi0_kernel_stats, e.g. "dcgs_update,dcgs_dots");
 * NULL or "" times every kernel.  Each timed launch adds two HIP events on
 * the stream, so timing only the kernels of interest keeps the overhead of
 * the events out of a measured run.  Resets the records; returns CHI0_OK,
 * or CHI0_EINVAL for a NULL context.  Valid on host-only contexts. */
int chi0_set_timing_filter(chi0_ctx *ctx, const char *names);

/*
 * Tile-shape autotuning of the dense matrix-core GEMMs (the virtual-orbital
 * transforms and the batched kernel product K V).  Enabled by default: the
 * first GEMM of a new shape class (kernel, M, K, split count, N within a half
 * octave) on a context times each valid tile variant (64x64, 64x128, 128x64,
 * 128x128 outputs per workgroup with k tiles of 16; 64x64 and 64x128 with k
 * tiles of 32) after a warm launch (the best of three timed launches), on the
 * call's stream, and keeps the fastest for that class.  All variants accumulate each
 * output element in the same order, so tuning never changes a result, only
 * the time; it does add a synchronisation of the stream on each new class.
 * chi0_set_autotune(ctx, mode): 1 tunes (default), 0 uses the 64x64 variant
 * everywhere, 100 + v forces variant v wherever it is valid for the shape
 * (64x64 elsewhere) without timing, for tests; other values: CHI0_EINVAL.
 * chi0_autotune_table copies up to `cap` entries of the context's table and
 * returns the number of entries (or a negative error code).
 */
typedef struct chi0_tune_record {
    char    key[96];      /* shape class */
    char    tile[16];     /* chosen variant, e.g. "64x128" */
    int32_t variant;      /* its index 0..5 */
    float   us[8];        /* timed launch of each variant in microseconds; 0 = not valid for the
                             shape (or beyond the library's variants) */
} chi0_tune_record;

int chi0_set_autotune(chi0_ctx *ctx, int32_t mode);
int chi0_autotune_table(chi0_ctx *ctx, chi0_tune_record *records, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* CHI0_H */
