// Host runtime of libchi0: the C-ABI declared in include/chi0.h.
//
// set_system validates the molecule, builds the atom-pair block maps of the
// sparse vertex (Sec. 3) and uploads padded device copies.  apply runs the
// matrix-free chi0(w) z sequence of Sec. 4.2 on a batch of vectors.
// solve_response drives GMRES (Sec. 4.1) for many (frequency, drive) points
// concurrently: each point owns a slot (Krylov basis, Hessenberg matrix,
// solution); every step applies the operator to one vector per active slot
// in a single batched pass, and a slot is refilled with the next point as
// soon as its point converges, so the batched transforms stay full.
#include "common.h"
#include "chi0.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace chi0;

// ================================================================== tracing
struct chi0::Tracer {
    bool on = false;
    struct Pending { const char *name; hipEvent_t a, b; double flops, bytes; };
    struct Rec { int64_t launches = 0; double ms = 0.0, flops = 0.0, bytes = 0.0; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, Rec> recs;
    std::vector<std::string> only;   // kernels to time; empty = all
    const char *cur_name = nullptr;
    hipEvent_t cur_a = nullptr;

    bool wanted(const char *name) const {
        if (only.empty()) return true;
        for (const auto &n : only)
            if (n == name) return true;
        return false;
    }

    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void harvest() {
        for (auto &p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                auto &r = recs[p.name];
                r.launches += 1;
                r.ms += ms;
                r.flops += p.flops;
                r.bytes += p.bytes;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    void clear() {
        harvest();
        recs.clear();
    }
    ~Tracer() {
        harvest();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

void chi0::trace_begin(Tracer *t, const char *name, hipStream_t s) {
    if (!t || !t->on) return;
    if (!t->wanted(name)) {
        t->cur_a = nullptr;
        return;
    }
    t->cur_name = name;
    t->cur_a = t->get();
    if (t->cur_a) (void)hipEventRecord(t->cur_a, s);
}

void chi0::trace_end(Tracer *t, hipStream_t s, double flops, double bytes) {
    if (!t || !t->on || !t->cur_a) return;
    hipEvent_t b = t->get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    t->pending.push_back({t->cur_name, t->cur_a, b, flops, bytes});
    t->cur_a = nullptr;
    if (t->pending.size() >= 16384) t->harvest();
}

// ================================================================== context
struct DevBuf {
    std::vector<void *> ptrs;
    void release() {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

// Buffers of one chi0 pass over up to nc_cap real columns (and its FP32
// intermediates for the low-precision operator, allocated on first use).
// chi0_apply uses op[0]; the solver gives each lane of slots its own.
struct OpWork {
    DevBuf buf, lpbuf;
    int nc_cap = 0, lp_cap = 0;
    double *Vb = nullptr, *Zin = nullptr, *Yout = nullptr, *dV = nullptr, *W = nullptr;
    double *Tt = nullptr, *at = nullptr, *Ut = nullptr, *part = nullptr, *omega_dev = nullptr;
    double *gemm_scratch = nullptr;
    size_t gemm_scratch_n = 0;
    float *Tt32 = nullptr, *at32 = nullptr, *Ut32 = nullptr;
    uint16_t *Bhi = nullptr, *Blo = nullptr;   // split-BF16 planes of the dense GEMMs' B operand
    void release() {
        lpbuf.release();
        buf.release();
        nc_cap = lp_cap = 0;
        Tt32 = at32 = Ut32 = nullptr;
        Bhi = Blo = nullptr;
    }
};
constexpr int kLanes = 4;            // most slot lanes of the solver, one stream each
constexpr int kAutoLanes = 2;        // lanes when the caller leaves the choice to the library
constexpr int kSets = 2 * kLanes;    // step buffer sets: two steps in flight per lane


struct chi0_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;
    Tracer tracer;
    GemmTuner tuner;

    // system
    bool has_system = false;
    int n_atoms = 0, N = 0, No = 0, Nv = 0, P = 0;
    int N_pad = 0, No_pad = 0, Nv_pad = 0, P_pad = 0;
    // the orbital counts rounded to the 16 of an MFMA k step: the extents the dense
    // transforms and the occupied sum of (b4) run over (the buffers keep the padding)
    int N16 = 0, No16 = 0, Nv16 = 0;
    double occ = 2.0;
    int n_blk = 0, n_g = 0, max_rows = 0, max_nprod = 0;
    int64_t nnzB = 0, npart = 0;
    WorkSizes ws{};
    DevBuf sysbuf;
    double *Xo = nullptr, *Xv = nullptr, *Xvt = nullptr, *Dlt = nullptr, *K = nullptr;
    BlockMapDev bm{};

    // operator workspaces (lane 0 also serves chi0_apply) and the lanes' streams
    OpWork op[kLanes];
    hipStream_t lane_stream[kLanes] = {};   // [0] is `stream`
    // chi0_apply as a HIP graph (chi0_set_graphs): the launch sequence of one
    // call, captured on cap_stream the second time a call repeats (the first
    // one runs eagerly and tunes the GEMM tiles), then replayed while the
    // call's rows, precision, buffers and broadening repeat.  Dropped whenever
    // the workspaces or the system are reallocated.
    struct ApplyKey {
        int nb = -1, prec = -1;
        const double *z = nullptr;
        double *out = nullptr;
        double eps = 0.0;
        bool operator==(const ApplyKey &o) const {
            return nb == o.nb && prec == o.prec && z == o.z && out == o.out && eps == o.eps;
        }
    };
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t apply_exec = nullptr;
    ApplyKey apply_key, apply_seen;
    void drop_apply_graph() {
        if (apply_exec) (void)hipGraphExecDestroy(apply_exec);
        apply_exec = nullptr;
        apply_key = ApplyKey{};
        apply_seen = ApplyKey{};
    }
    // low-precision operator: operand copies (set_system)
    float *Xo32 = nullptr, *Xv32 = nullptr, *Xvt32 = nullptr;
    uint16_t *Xv_hi = nullptr, *Xv_lo = nullptr, *Xvt_hi = nullptr, *Xvt_lo = nullptr;

    // partial reorthogonalisation with kernel timing on: per step, whether the
    // pass ran and the b_j (one per drive) that the device decision used
    std::vector<int32_t> lz_pass_rec;
    std::vector<double> lz_bpre_rec;

    // solver workspace
    DevBuf slotbuf;
    int slot_n = 0, slot_m = 0;
    SlotsDev slots{};
    // kSets sets of step buffers (two steps in flight per lane).  Set q of the
    // job arena holds [Job x slot_n][double omega x slot_n], so one copy moves
    // a step's jobs and frequencies; fin/upd/status are [kSets][slot_n].
    char *arena_dev = nullptr, *arena_h = nullptr;
    Job *fin_dev = nullptr, *upd_dev = nullptr;
    StepStatus *status_dev = nullptr;
    Job *fin_h = nullptr, *upd_h = nullptr;
    StepStatus *status_h = nullptr;
    int host_cap = 0;
    hipEvent_t step_ev[kSets] = {};
    size_t arena_bytes() const { return (size_t)slot_n * (sizeof(Job) + sizeof(double)); }
    Job *jobs_dev(int q) { return reinterpret_cast<Job *>(arena_dev + q * arena_bytes()); }
    double *somega_dev(int q) { return reinterpret_cast<double *>(arena_dev + q * arena_bytes() + slot_n * sizeof(Job)); }
    Job *jobs_h(int q) { return reinterpret_cast<Job *>(arena_h + q * arena_bytes()); }
    double *omega_h(int q) { return reinterpret_cast<double *>(arena_h + q * arena_bytes() + slot_n * sizeof(Job)); }

    ~chi0_ctx() {
        if (device >= 0) {
            (void)hipSetDevice(device);
            if (stream) (void)hipStreamSynchronize(stream);
        }
        if (device >= 0)
            for (hipStream_t ls : lane_stream)
                if (ls) (void)hipStreamSynchronize(ls);
        slotbuf.release();
        for (OpWork &o : op) o.release();
        sysbuf.release();
        if (arena_h) (void)hipHostFree(arena_h);
        if (fin_h) (void)hipHostFree(fin_h);
        if (upd_h) (void)hipHostFree(upd_h);
        if (status_h) (void)hipHostFree(status_h);
        for (hipEvent_t &e : step_ev)
            if (e) (void)hipEventDestroy(e);
        for (int L = 1; L < kLanes; ++L)
            if (lane_stream[L]) (void)hipStreamDestroy(lane_stream[L]);
        drop_apply_graph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

static thread_local std::string g_create_error;

static int fail(chi0_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, e_ == hipErrorOutOfMemory ? CHI0_ENOMEM : CHI0_EHIP,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));                \
    } while (0)

template <class T>
static int dalloc(chi0_ctx *c, DevBuf &buf, T **p, int64_t n) {
    void *q = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess)
        return fail(c, CHI0_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                        hipGetErrorString(e));
    buf.ptrs.push_back(q);
    // The zero fill runs on the null stream, which is not ordered with the
    // context's non-blocking streams: wait for it, so that work enqueued on
    // those streams after dalloc returns never races with the fill.
    e = hipMemset(q, 0, bytes);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return fail(c, CHI0_EHIP, std::string("hipMemset: ") + hipGetErrorString(e));
    *p = static_cast<T *>(q);
    return CHI0_OK;
}

#define CHK(x)                      \
    do {                            \
        int r_ = (x);               \
        if (r_ != CHI0_OK) return r_; \
    } while (0)

// ============================================================ static scratch
// Workspace of chi0_apply_noalloc: a fixed array in device memory, one copy
// per GPU, held until the process ends.  Host code never uses the array's
// name as an address; chi0_create looks up each device's copy once (with
// that device current) and the entry point passes that address to kernels.
constexpr int64_t kScratchDoubles = CHI0_NOALLOC_SCRATCH_BYTES / 8;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static double *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Address of `scratch` on the current device `device` (looked up on the first call).
static hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

// ================================================================ lifecycle
extern "C" int chi0_create(chi0_ctx **out, int device) {
    if (!out) { g_create_error = "out is NULL"; return CHI0_EINVAL; }
    *out = nullptr;
    if (device < -1) { g_create_error = "device must be >= -1"; return CHI0_EINVAL; }
    chi0_ctx *c = new (std::nothrow) chi0_ctx();
    if (!c) { g_create_error = "out of host memory"; return CHI0_ENOMEM; }
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            g_create_error = "HIP device " + std::to_string(device) + " not available (" +
                             std::to_string(e == hipSuccess ? n : 0) + " devices)";
            delete c;
            return e == hipSuccess ? CHI0_EINVAL : CHI0_EHIP;
        }
        e = hipSetDevice(device);
        if (e == hipSuccess) e = scratch_setup(device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        for (int L = 1; L < kLanes && e == hipSuccess; ++L)
            e = hipStreamCreateWithFlags(&c->lane_stream[L], hipStreamNonBlocking);
        c->lane_stream[0] = c->stream;
        if (e != hipSuccess) {
            g_create_error = std::string("HIP setup failed: ") + hipGetErrorString(e);
            delete c;
            return CHI0_EHIP;
        }
        c->device = device;
    }
    *out = c;
    return CHI0_OK;
}

extern "C" void chi0_destroy(chi0_ctx *ctx) { delete ctx; }

extern "C" const char *chi0_last_error(const chi0_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

extern "C" int chi0_get_sizes(const chi0_ctx *ctx, int32_t *n_orb, int32_t *n_occ,
                              int32_t *n_prod, int32_t *n_atoms) {
    if (!ctx) return CHI0_EINVAL;
    if (!ctx->has_system) return CHI0_ENOSYS;
    if (n_orb) *n_orb = ctx->N;
    if (n_occ) *n_occ = ctx->No;
    if (n_prod) *n_prod = ctx->P;
    if (n_atoms) *n_atoms = ctx->n_atoms;
    return CHI0_OK;
}

extern "C" void chi0_solve_opts_default(chi0_solve_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->restart = 30;
    o->max_iter = 10000;
    o->tol = 1e-10;
    o->precision = CHI0_PREC_FP64;
    o->batch = 1;
}

extern "C" int chi0_set_timing(chi0_ctx *ctx, int32_t enable) {
    if (!ctx) return CHI0_EINVAL;
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    ctx->tracer.clear();
    ctx->tracer.on = enable != 0;
    return CHI0_OK;
}

extern "C" int chi0_set_timing_filter(chi0_ctx *ctx, const char *names) {
    if (!ctx) return CHI0_EINVAL;
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    ctx->tracer.clear();
    ctx->tracer.only.clear();
    if (names) {
        std::string cur;
        for (const char *p = names;; ++p) {
            if (*p == ',' || *p == '\0') {
                if (!cur.empty()) ctx->tracer.only.push_back(cur);
                cur.clear();
                if (*p == '\0') break;
            } else if (*p != ' ') {
                cur.push_back(*p);
            }
        }
    }
    return CHI0_OK;
}

extern "C" int chi0_set_autotune(chi0_ctx *ctx, int32_t mode) {
    if (!ctx) return CHI0_EINVAL;
    if (mode >= 100 && mode < 100 + GEMM_VARIANTS) {
        ctx->tuner.force = mode - 100;
        return CHI0_OK;
    }
    if (mode != 0 && mode != 1) return fail(ctx, CHI0_EINVAL, "autotune mode must be 0, 1 or 100 + variant");
    ctx->tuner.force = -1;
    ctx->tuner.enabled = mode != 0;
    return CHI0_OK;
}

extern "C" int chi0_autotune_table(chi0_ctx *ctx, chi0_tune_record *rec, int32_t cap) {
    if (!ctx || cap < 0 || (cap > 0 && !rec)) return fail(ctx, CHI0_EINVAL, "bad arguments");
    int i = 0;
    for (auto &kv : ctx->tuner.table) {
        if (i < cap) {
            std::memset(&rec[i], 0, sizeof(rec[i]));
            std::snprintf(rec[i].key, sizeof(rec[i].key), "%s", kv.first.c_str());
            rec[i].variant = kv.second.variant;
            std::snprintf(rec[i].tile, sizeof(rec[i].tile), "%s", kGemmVariantNames[kv.second.variant]);
            for (int v = 0; v < GEMM_VARIANTS && v < 8; ++v) rec[i].us[v] = kv.second.us[v];
        }
        ++i;
    }
    return i;
}

extern "C" int chi0_kernel_stats(chi0_ctx *ctx, chi0_kernel_record *rec, int32_t cap) {
    if (!ctx || cap < 0 || (cap > 0 && !rec)) return fail(ctx, CHI0_EINVAL, "bad arguments");
    if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
    ctx->tracer.harvest();
    int i = 0;
    for (auto &kv : ctx->tracer.recs) {
        if (i < cap) {
            std::memset(&rec[i], 0, sizeof(rec[i]));
            std::snprintf(rec[i].name, sizeof(rec[i].name), "%s", kv.first.c_str());
            rec[i].launches = kv.second.launches;
            rec[i].total_ms = kv.second.ms;
            rec[i].flops = kv.second.flops;
            rec[i].bytes = kv.second.bytes;
        }
        ++i;
    }
    return i;
}

// =============================================================== set_system
namespace {

struct HostMaps {
    std::vector<int32_t> blk_nprod, blk_na, blk_nb, pidx, col_gstart, g_xrow, atom_off;
    std::vector<int64_t> blk_pstart, blk_vstart, blk_ent, g_ent, prod_pstart, prod_plist;
    std::vector<double> Vp;
    int max_rows = 0;
};

bool all_finite(const double *p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

static void drop_system(chi0_ctx *c) {
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
    }
    for (hipStream_t ls : c->lane_stream)
        if (c->device >= 0 && ls) (void)hipStreamSynchronize(ls);
    c->slotbuf.release();
    c->slot_n = c->slot_m = 0;
    c->drop_apply_graph();
    for (OpWork &o : c->op) o.release();
    c->sysbuf.release();
    c->has_system = false;
}

extern "C" int chi0_set_system(chi0_ctx *c, int32_t n_atoms, const double *positions,
                               int32_t n_orb, int32_t n_occ, double occ_factor,
                               const double *eig, const double *X, const int32_t *aoff,
                               int32_t n_prod, const int32_t *pat, const int64_t *voff,
                               const double *vblock, const double *K) {
    if (!c) return CHI0_EINVAL;
    drop_system(c);
    // ---------------------------------------------------------- validation
    if (n_atoms < 1 || n_orb < 2 || n_occ < 1 || n_occ >= n_orb || n_prod < 1)
        return fail(c, CHI0_EINVAL, "need n_atoms >= 1, n_orb >= 2, 1 <= n_occ < n_orb, n_prod >= 1");
    if (!eig || !X || !aoff || !pat || !voff || !vblock || !K)
        return fail(c, CHI0_EINVAL, "NULL input pointer");
    if (!(occ_factor > 0.0) || !std::isfinite(occ_factor))
        return fail(c, CHI0_EINVAL, "occ_factor must be finite and > 0");
    if (aoff[0] != 0 || aoff[n_atoms] != n_orb)
        return fail(c, CHI0_EINVAL, "atom_orb_offset must start at 0 and end at n_orb");
    for (int A = 0; A < n_atoms; ++A) {
        const int na = aoff[A + 1] - aoff[A];
        if (na < 1) return fail(c, CHI0_EINVAL, "atom_orb_offset must be strictly increasing");
        if (na > NB_MAX)
            return fail(c, CHI0_EINVAL, "atom " + std::to_string(A) + " has " + std::to_string(na) +
                                            " orbitals; at most " + std::to_string(NB_MAX) + " supported");
    }
    std::vector<int> s_mu(n_prod);
    for (int mu = 0; mu < n_prod; ++mu) {
        const int A = pat[2 * mu], B = pat[2 * mu + 1];
        if (A < 0 || A >= n_atoms || B < -1 || B >= n_atoms || B == A)
            return fail(c, CHI0_EINVAL, "bad prod_atoms entry for product " + std::to_string(mu));
        s_mu[mu] = (aoff[A + 1] - aoff[A]) + (B >= 0 ? aoff[B + 1] - aoff[B] : 0);
    }
    if (voff[0] != 0) return fail(c, CHI0_EINVAL, "vblock_offset[0] must be 0");
    for (int mu = 0; mu < n_prod; ++mu)
        if (voff[mu + 1] - voff[mu] != (int64_t)s_mu[mu] * s_mu[mu])
            return fail(c, CHI0_EINVAL, "vblock_offset of product " + std::to_string(mu) +
                                            " does not match its support size");
    const int64_t nv_tot = voff[n_prod];
    if (positions && !all_finite(positions, 3 * (int64_t)n_atoms))
        return fail(c, CHI0_ENONFINITE, "non-finite positions");
    if (!all_finite(eig, n_orb)) return fail(c, CHI0_ENONFINITE, "non-finite eigenvalues");
    if (!all_finite(X, (int64_t)n_orb * n_orb)) return fail(c, CHI0_ENONFINITE, "non-finite X");
    if (!all_finite(vblock, nv_tot)) return fail(c, CHI0_ENONFINITE, "non-finite vertex");
    if (!all_finite(K, (int64_t)n_prod * n_prod)) return fail(c, CHI0_ENONFINITE, "non-finite K");
    for (int E = 0; E < n_orb; ++E) {
        if (E < n_occ && !(eig[E] < 0.0))
            return fail(c, CHI0_EINVAL, "occupied eigenvalues must be < 0 (energies shifted to the gap)");
        if (E >= n_occ && !(eig[E] > 0.0))
            return fail(c, CHI0_EINVAL, "virtual eigenvalues must be > 0 (energies shifted to the gap)");
    }
    for (int mu = 0; mu < n_prod; ++mu) {
        const int s = s_mu[mu];
        const double *b = vblock + voff[mu];
        double mx = 0.0;
        for (int i = 0; i < s * s; ++i) mx = std::max(mx, std::fabs(b[i]));
        for (int i = 0; i < s; ++i)
            for (int j = i + 1; j < s; ++j)
                if (std::fabs(b[i * s + j] - b[j * s + i]) > 1e-12 * mx)
                    return fail(c, CHI0_EASYM, "vertex block of product " + std::to_string(mu) + " is not symmetric");
    }
    {
        double mx = 0.0;
        for (int64_t i = 0; i < (int64_t)n_prod * n_prod; ++i) mx = std::max(mx, std::fabs(K[i]));
        for (int i = 0; i < n_prod; ++i)
            for (int j = i + 1; j < n_prod; ++j)
                if (std::fabs(K[(int64_t)i * n_prod + j] - K[(int64_t)j * n_prod + i]) > 1e-12 * mx)
                    return fail(c, CHI0_EASYM, "kernel matrix K is not symmetric");
    }

    // ------------------------------------------------------- block maps
    HostMaps hm;
    hm.atom_off.assign(aoff, aoff + n_atoms + 1);
    std::map<std::pair<int, int>, int> blk_of;
    std::vector<std::pair<int, int>> blocks;
    for (int A = 0; A < n_atoms; ++A) { blk_of[{A, A}] = (int)blocks.size(); blocks.push_back({A, A}); }
    {
        std::vector<std::pair<int, int>> offd;
        for (int mu = 0; mu < n_prod; ++mu)
            if (pat[2 * mu + 1] >= 0) {
                const int A = pat[2 * mu], B = pat[2 * mu + 1];
                offd.push_back({A, B});
                offd.push_back({B, A});
            }
        std::sort(offd.begin(), offd.end());
        offd.erase(std::unique(offd.begin(), offd.end()), offd.end());
        for (auto &ab : offd) { blk_of[ab] = (int)blocks.size(); blocks.push_back(ab); }
    }
    const int nblk = (int)blocks.size();
    struct Ent { int mu, ro, co; };
    std::vector<std::vector<Ent>> ents(nblk);
    for (int mu = 0; mu < n_prod; ++mu) {
        const int A = pat[2 * mu], B = pat[2 * mu + 1];
        const int na = aoff[A + 1] - aoff[A];
        ents[blk_of[{A, A}]].push_back({mu, 0, 0});
        if (B >= 0) {
            ents[blk_of[{A, B}]].push_back({mu, 0, na});
            ents[blk_of[{B, A}]].push_back({mu, na, 0});
            ents[blk_of[{B, B}]].push_back({mu, na, na});
        }
    }
    hm.blk_nprod.resize(nblk); hm.blk_na.resize(nblk); hm.blk_nb.resize(nblk);
    hm.blk_pstart.resize(nblk); hm.blk_vstart.resize(nblk); hm.blk_ent.resize(nblk);
    std::vector<std::vector<int64_t>> pos_of(n_prod);
    int64_t pcur = 0, vcur = 0, ecur = 0;
    for (int k = 0; k < nblk; ++k) {
        const int A = blocks[k].first, B = blocks[k].second;
        const int na = aoff[A + 1] - aoff[A], nb = aoff[B + 1] - aoff[B];
        hm.blk_na[k] = na; hm.blk_nb[k] = nb;
        hm.blk_nprod[k] = (int)ents[k].size();
        hm.blk_pstart[k] = pcur; hm.blk_vstart[k] = vcur; hm.blk_ent[k] = ecur;
        for (auto &e : ents[k]) {
            const int s = s_mu[e.mu];
            const double *b = vblock + voff[e.mu];
            for (int a = 0; a < na; ++a)
                for (int bb = 0; bb < nb; ++bb) hm.Vp.push_back(b[(e.ro + a) * s + e.co + bb]);
            hm.pidx.push_back(e.mu);
            pos_of[e.mu].push_back(pcur);
            ++pcur;
            vcur += (int64_t)na * nb;
        }
        ecur += (int64_t)na * nb;
    }
    hm.prod_pstart.resize(n_prod + 1);
    hm.prod_pstart[0] = 0;
    for (int mu = 0; mu < n_prod; ++mu) {
        for (auto p : pos_of[mu]) hm.prod_plist.push_back(p);
        hm.prod_pstart[mu + 1] = (int64_t)hm.prod_plist.size();
    }
    // gathered rows per column atom B: rows (A, a) over blocks (A, B), A ascending
    std::vector<std::vector<int>> col_blocks(n_atoms);
    for (int k = 0; k < nblk; ++k) col_blocks[blocks[k].second].push_back(k);
    hm.col_gstart.resize(n_atoms + 1);
    for (int B = 0; B < n_atoms; ++B) {
        auto &cb = col_blocks[B];
        std::sort(cb.begin(), cb.end(), [&](int x, int y) { return blocks[x].first < blocks[y].first; });
        hm.col_gstart[B] = (int32_t)hm.g_xrow.size();
        const int nb = aoff[B + 1] - aoff[B];
        for (int k : cb) {
            const int A = blocks[k].first, na = aoff[A + 1] - aoff[A];
            for (int a = 0; a < na; ++a) {
                hm.g_xrow.push_back(aoff[A] + a);
                hm.g_ent.push_back(hm.blk_ent[k] + (int64_t)a * nb);
            }
        }
        hm.max_rows = std::max(hm.max_rows, (int)hm.g_xrow.size() - hm.col_gstart[B]);
    }
    hm.col_gstart[n_atoms] = (int32_t)hm.g_xrow.size();

    c->n_atoms = n_atoms; c->N = n_orb; c->No = n_occ; c->Nv = n_orb - n_occ; c->P = n_prod;
    c->N_pad = (int)round_up(n_orb, TILE);
    c->No_pad = (int)round_up(n_occ, TILE);
    c->Nv_pad = (int)round_up(n_orb - n_occ, TILE);
    c->P_pad = (int)round_up(n_prod, TILE);
    c->N16 = (int)round_up(n_orb, 16);
    c->No16 = (int)round_up(n_occ, 16);
    c->Nv16 = (int)round_up(n_orb - n_occ, 16);
    c->occ = occ_factor;
    c->n_blk = nblk; c->n_g = (int)hm.g_xrow.size(); c->max_rows = hm.max_rows;
    c->max_nprod = *std::max_element(hm.blk_nprod.begin(), hm.blk_nprod.end());
    c->nnzB = ecur; c->npart = pcur;
    c->ws.N = n_orb; c->ws.No = n_occ; c->ws.Nv = n_orb - n_occ; c->ws.P = n_prod;
    c->ws.nnzB = (double)ecur; c->ws.npart = (double)pcur; c->ws.sum_s2 = (double)nv_tot;

    if (c->device < 0) {   // host-only context: validation and maps only
        c->has_system = true;
        c->err.clear();
        return CHI0_OK;
    }
    HIPCHK(c, hipSetDevice(c->device));

    // ------------------------------------------------------------ upload
    const int N = n_orb, No = n_occ, Nv = n_orb - n_occ;
    DevBuf &sb = c->sysbuf;
    {
        std::vector<double> xo((size_t)c->N_pad * c->No_pad, 0.0), xv((size_t)c->N_pad * c->Nv_pad, 0.0),
            xvt((size_t)c->Nv_pad * c->N_pad, 0.0), dl((size_t)c->No_pad * c->Nv_pad, 1.0);
        for (int a = 0; a < N; ++a) {
            for (int E = 0; E < No; ++E) xo[(size_t)a * c->No_pad + E] = X[(size_t)a * N + E];
            for (int F = 0; F < Nv; ++F) {
                xv[(size_t)a * c->Nv_pad + F] = X[(size_t)a * N + No + F];
                xvt[(size_t)F * c->N_pad + a] = X[(size_t)a * N + No + F];
            }
        }
        for (int E = 0; E < No; ++E)
            for (int F = 0; F < Nv; ++F) dl[(size_t)E * c->Nv_pad + F] = eig[No + F] - eig[E];
        CHK(dalloc(c, sb, &c->Xo, (int64_t)xo.size()));
        CHK(dalloc(c, sb, &c->Xv, (int64_t)xv.size()));
        CHK(dalloc(c, sb, &c->Xvt, (int64_t)xvt.size()));
        CHK(dalloc(c, sb, &c->Dlt, (int64_t)dl.size()));
        HIPCHK(c, hipMemcpy(c->Xo, xo.data(), xo.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->Xv, xv.data(), xv.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->Xvt, xvt.data(), xvt.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->Dlt, dl.data(), dl.size() * 8, hipMemcpyHostToDevice));
        // operand copies of the low-precision operator
        CHK(dalloc(c, sb, &c->Xo32, (int64_t)xo.size()));
        CHK(dalloc(c, sb, &c->Xv32, (int64_t)xv.size()));
        CHK(dalloc(c, sb, &c->Xvt32, (int64_t)xvt.size()));
        CHK(dalloc(c, sb, &c->Xv_hi, (int64_t)xv.size()));
        CHK(dalloc(c, sb, &c->Xv_lo, (int64_t)xv.size()));
        CHK(dalloc(c, sb, &c->Xvt_hi, (int64_t)xvt.size()));
        CHK(dalloc(c, sb, &c->Xvt_lo, (int64_t)xvt.size()));
        HIPCHK(c, hipDeviceSynchronize());
        launch_to_f32(nullptr, c->Xo, c->Xo32, (int64_t)xo.size());
        launch_to_f32(nullptr, c->Xv, c->Xv32, (int64_t)xv.size());
        launch_to_f32(nullptr, c->Xvt, c->Xvt32, (int64_t)xvt.size());
        launch_split_bf16(nullptr, c->Xv, c->Xv_hi, c->Xv_lo, (int64_t)xv.size());
        launch_split_bf16(nullptr, c->Xvt, c->Xvt_hi, c->Xvt_lo, (int64_t)xvt.size());
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipDeviceSynchronize());
    }
    CHK(dalloc(c, sb, &c->K, (int64_t)c->P_pad * c->P_pad));
    HIPCHK(c, hipMemcpy2D(c->K, (size_t)c->P_pad * 8, K, (size_t)n_prod * 8, (size_t)n_prod * 8,
                          (size_t)n_prod, hipMemcpyHostToDevice));

    auto up32 = [&](const std::vector<int32_t> &v, const int32_t **dst) -> int {
        int32_t *p = nullptr;
        CHK(dalloc(c, sb, &p, (int64_t)v.size()));
        if (!v.empty()) HIPCHK(c, hipMemcpy(p, v.data(), v.size() * 4, hipMemcpyHostToDevice));
        *dst = p;
        return CHI0_OK;
    };
    auto up64 = [&](const std::vector<int64_t> &v, const int64_t **dst) -> int {
        int64_t *p = nullptr;
        CHK(dalloc(c, sb, &p, (int64_t)v.size()));
        if (!v.empty()) HIPCHK(c, hipMemcpy(p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
        *dst = p;
        return CHI0_OK;
    };
    BlockMapDev &bm = c->bm;
    CHK(up32(hm.blk_nprod, &bm.blk_nprod));
    CHK(up64(hm.blk_pstart, &bm.blk_pstart));
    CHK(up64(hm.blk_vstart, &bm.blk_vstart));
    CHK(up64(hm.blk_ent, &bm.blk_ent));
    CHK(up32(hm.blk_na, &bm.blk_na));
    CHK(up32(hm.blk_nb, &bm.blk_nb));
    CHK(up32(hm.pidx, &bm.pidx));
    CHK(up32(hm.col_gstart, &bm.col_gstart));
    CHK(up32(hm.g_xrow, &bm.g_xrow));
    CHK(up64(hm.g_ent, &bm.g_ent));
    CHK(up32(hm.atom_off, &bm.atom_off));
    bm.nb_max = 0;
    for (size_t A = 0; A + 1 < hm.atom_off.size(); ++A)
        bm.nb_max = std::max(bm.nb_max, hm.atom_off[A + 1] - hm.atom_off[A]);
    CHK(up64(hm.prod_pstart, &bm.prod_pstart));
    CHK(up64(hm.prod_plist, &bm.prod_plist));
    {
        double *vp = nullptr;
        CHK(dalloc(c, sb, &vp, (int64_t)hm.Vp.size()));
        HIPCHK(c, hipMemcpy(vp, hm.Vp.data(), hm.Vp.size() * 8, hipMemcpyHostToDevice));
        bm.Vp = vp;
    }
    HIPCHK(c, hipDeviceSynchronize());
    c->has_system = true;
    c->err.clear();
    return CHI0_OK;
}

// ================================================================ operator
static int ensure_ws(chi0_ctx *c, OpWork &o, int nc) {
    if (nc <= o.nc_cap) return CHI0_OK;
    for (hipStream_t ls : c->lane_stream)
        if (ls) HIPCHK(c, hipStreamSynchronize(ls));
    HIPCHK(c, hipDeviceSynchronize());
    c->drop_apply_graph();
    o.release();
    DevBuf &w = o.buf;
    const int64_t mcol = (int64_t)c->No_pad * nc;
    CHK(dalloc(c, w, &o.Vb, (int64_t)c->P_pad * nc));
    CHK(dalloc(c, w, &o.Zin, (int64_t)c->P_pad * nc));
    CHK(dalloc(c, w, &o.Yout, (int64_t)c->P_pad * nc));
    CHK(dalloc(c, w, &o.dV, c->nnzB * nc));
    CHK(dalloc(c, w, &o.W, c->nnzB * nc));
    CHK(dalloc(c, w, &o.Tt, (int64_t)c->N_pad * mcol));
    CHK(dalloc(c, w, &o.Ut, (int64_t)c->N_pad * mcol));
    CHK(dalloc(c, w, &o.at, (int64_t)c->Nv_pad * mcol));
    CHK(dalloc(c, w, &o.part, c->npart * nc));
    CHK(dalloc(c, w, &o.omega_dev, nc / 2 + 1));
    // split-K partials: splits are only used while tiles * splits < 2048, so
    // the partial products never exceed 2048 64x64 tiles
    o.gemm_scratch_n = (size_t)2048 * 64 * 64;
    CHK(dalloc(c, w, &o.gemm_scratch, (int64_t)o.gemm_scratch_n));
    HIPCHK(c, hipDeviceSynchronize());
    o.nc_cap = nc;
    return CHI0_OK;
}

static int ensure_lp(chi0_ctx *c, OpWork &o) {
    if (o.lp_cap >= o.nc_cap && o.Tt32) return CHI0_OK;
    for (hipStream_t ls : c->lane_stream)
        if (ls) HIPCHK(c, hipStreamSynchronize(ls));
    HIPCHK(c, hipDeviceSynchronize());
    c->drop_apply_graph();
    o.lpbuf.release();
    o.lp_cap = 0;
    const int64_t mcol = (int64_t)c->No_pad * o.nc_cap;
    CHK(dalloc(c, o.lpbuf, &o.Tt32, (int64_t)c->N_pad * mcol));
    CHK(dalloc(c, o.lpbuf, &o.Ut32, (int64_t)c->N_pad * mcol));
    CHK(dalloc(c, o.lpbuf, &o.at32, (int64_t)c->Nv_pad * mcol));
    // two uint16 planes of max(N_pad, Nv_pad) x mcol: as many bytes as one FP32 copy
    const int64_t kmax = std::max(c->N_pad, c->Nv_pad);
    double *planes = nullptr;
    CHK(dalloc(c, o.lpbuf, &planes, (kmax * mcol + 3) / 4 * 2));
    o.Bhi = reinterpret_cast<uint16_t *>(planes);
    o.Blo = o.Bhi + (kmax * mcol + 3) / 4 * 4;
    HIPCHK(c, hipDeviceSynchronize());
    o.lp_cap = o.nc_cap;
    return CHI0_OK;
}

// Y = chi0(omega) Zin for nb column pairs already in Zin; omega: device [nb].
// prec selects the arithmetic of the orbital transforms (ensure_lp first).
// t, tu: the tracer and GEMM tuner to use (the context's; NULL for none).
static void run_chi0(chi0_ctx *c, OpWork &o, hipStream_t s, int nb, double eps, int prec,
                     const double *omega, Tracer *t, GemmTuner *tu) {
    const int nc = 2 * nb;
    const WorkSizes &w = c->ws;
    const int64_t mcol = (int64_t)c->No_pad * nc;
    // the dense transforms' columns (E, j) for E < No16 and sums over k < N16 / Nv16:
    // the rest of the padded layout holds zeros and is not multiplied
    const int ncol = c->No16 * nc;
    // algorithmic work of the two dense transforms (unpadded sizes)
    const double fl = 2.0 * w.N * w.Nv * w.No * nc;
    launch_vertex_gather(t, s, c->bm, c->n_blk, o.Zin, o.dV, nc, w);
    if (prec == CHI0_PREC_FP64) {
        launch_occ_transform(t, s, c->bm, c->n_atoms, c->Xo, c->No_pad, o.dV, o.Tt, nc, w);
        launch_dgemm_lorentz(t, s, c->Nv_pad, ncol, c->N16, c->N_pad, c->Xvt, c->N_pad, o.Tt, (int)mcol,
                             o.at, (int)mcol, c->Dlt, c->Nv_pad, omega, eps, c->occ, nc,
                             fl + 6.0 * w.No * w.Nv * nb,
                             8.0 * (w.N * w.No * nc + w.Nv * w.No * nc + w.N * w.Nv + w.No * w.Nv),
                             o.gemm_scratch, o.gemm_scratch_n, tu);
        launch_dgemm(t, s, "virt_back", c->N_pad, ncol, c->Nv16, c->Nv_pad, c->Xv, c->Nv_pad, o.at, (int)mcol,
                     o.Ut, (int)mcol, fl, 8.0 * (w.Nv * w.No * nc + w.N * w.No * nc + w.N * w.Nv),
                     o.gemm_scratch, o.gemm_scratch_n, tu);
        launch_occ_back(t, s, c->bm, c->n_atoms, c->max_rows, c->Xo, c->No_pad, c->No16, o.Ut, o.W, nc, w);
    } else {
        launch_occ_transform_f32(t, s, c->bm, c->n_atoms, c->Xo32, c->No_pad, o.dV, o.Tt32, nc, w);
        LorentzArgs la{c->Dlt, omega, c->Nv_pad, nc, eps, c->occ};
        const size_t sb = o.gemm_scratch_n * sizeof(double);
        const double by = 4.0 * (w.N * w.No * nc + w.Nv * w.No * nc);
        if (prec == CHI0_PREC_FP32) {
            launch_sgemm(t, s, "virt_transform_lorentz_f32", c->Nv_pad, ncol, c->N_pad, c->Xvt32,
                         c->N_pad, o.Tt32, (int)mcol, o.at32, (int)mcol, fl + 6.0 * w.No * w.Nv * nb,
                         by + 4.0 * w.N * w.Nv, &la, o.gemm_scratch, sb, tu);
            launch_sgemm(t, s, "virt_back_f32", c->N_pad, ncol, c->Nv_pad, c->Xv32, c->Nv_pad,
                         o.at32, (int)mcol, o.Ut32, (int)mcol, fl, by + 4.0 * w.N * w.Nv, nullptr,
                         o.gemm_scratch, sb, tu);
        } else {   // split BF16 x 3: three BF16 products per multiply-add
            launch_bgemm3(t, s, "virt_transform_lorentz_bf16x3", c->Nv_pad, ncol, c->N_pad, c->Xvt_hi,
                          c->Xvt_lo, c->N_pad, o.Tt32, (int)mcol, o.Bhi, o.Blo, o.at32, (int)mcol, 3.0 * fl,
                          by + 4.0 * w.N * w.Nv, &la, o.gemm_scratch, sb);
            launch_bgemm3(t, s, "virt_back_bf16x3", c->N_pad, ncol, c->Nv_pad, c->Xv_hi, c->Xv_lo,
                          c->Nv_pad, o.at32, (int)mcol, o.Bhi, o.Blo, o.Ut32, (int)mcol, 3.0 * fl,
                          by + 4.0 * w.N * w.Nv, nullptr, o.gemm_scratch, sb);
        }
        launch_occ_back_f32(t, s, c->bm, c->n_atoms, c->max_rows, c->Xo32, c->No_pad, c->No16, o.Ut32, o.W, nc, w);
    }
    launch_vertex_contract(t, s, c->bm, c->n_blk, c->P, o.W, o.part, o.Yout, nc, w, c->max_nprod);
}

static const int kMaxBatch = 256;   // complex columns per operator pass
// normwise relative error of one low-precision chi0 application (measured on
// the test systems: ~3e-7 with FP32 transforms, ~5-7e-6 with split BF16 x 3)
static const double kOpErrFP32 = 3e-7, kOpErrBF16X3 = 6e-6;

extern "C" int chi0_apply(chi0_ctx *c, int32_t n_rhs, const double *omega, double eps,
                          const double *z, double *out, int32_t precision, void *stream) {
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    if (n_rhs < 0) return fail(c, CHI0_EINVAL, "n_rhs < 0");
    if (n_rhs == 0) return CHI0_OK;
    if (!omega || !z || !out) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (precision < CHI0_PREC_FP64 || precision > CHI0_PREC_BF16X3)
        return fail(c, CHI0_EINVAL, "unknown precision");
    if (!all_finite(omega, n_rhs)) return fail(c, CHI0_ENONFINITE, "non-finite omega");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cap = std::min(kMaxBatch, std::max(n_rhs, 1));
    OpWork &ow = c->op[0];
    CHK(ensure_ws(c, ow, 2 * std::max(cap, ow.nc_cap / 2)));
    if (precision != CHI0_PREC_FP64) CHK(ensure_lp(c, ow));
    // graph replay: one operator pass (n_rhs <= cap), not traced
    if (c->graphs && n_rhs <= cap && !c->tracer.on) {
        chi0_ctx::ApplyKey k;
        k.nb = n_rhs;
        k.prec = precision;
        k.z = z;
        k.out = out;
        k.eps = eps;
        const int nc = 2 * n_rhs;
        if (!(c->apply_exec && c->apply_key == k) && c->apply_seen == k) {
            // second call with this key: capture its launch sequence
            c->drop_apply_graph();
            if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            launch_rows_to_cols(&c->tracer, c->cap_stream, z, n_rhs, c->P, ow.Zin, nc);
            run_chi0(c, ow, c->cap_stream, n_rhs, eps, precision, ow.omega_dev, &c->tracer, &c->tuner);
            launch_cols_to_rows(&c->tracer, c->cap_stream, ow.Yout, n_rhs, c->P, nc, out);
            HIPCHK(c, hipStreamEndCapture(c->cap_stream, &g));
            const hipError_t e = hipGraphInstantiate(&c->apply_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->apply_exec = nullptr;
                return fail(c, CHI0_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            c->apply_key = k;
        }
        if (c->apply_exec && c->apply_key == k) {
            HIPCHK(c, hipMemcpyAsync(ow.omega_dev, omega, (size_t)n_rhs * 8, hipMemcpyHostToDevice, s));
            HIPCHK(c, hipGraphLaunch(c->apply_exec, s));
            return CHI0_OK;
        }
        c->apply_seen = k;   // first call with this key: eager (tunes the GEMM tiles)
    }
    for (int r0 = 0; r0 < n_rhs; r0 += cap) {
        const int nb = std::min(cap, n_rhs - r0), nc = 2 * nb;
        HIPCHK(c, hipMemcpyAsync(ow.omega_dev, omega + r0, (size_t)nb * 8, hipMemcpyHostToDevice, s));
        launch_rows_to_cols(&c->tracer, s, z + (int64_t)r0 * c->P * 2, nb, c->P, ow.Zin, nc);
        run_chi0(c, ow, s, nb, eps, precision, ow.omega_dev, &c->tracer, &c->tuner);
        launch_cols_to_rows(&c->tracer, s, ow.Yout, nb, c->P, nc, out + (int64_t)r0 * c->P * 2);
    }
    HIPCHK(c, hipGetLastError());
    return CHI0_OK;
}

extern "C" int chi0_set_graphs(chi0_ctx *c, int32_t enable) {
    if (!c) return CHI0_EINVAL;
    if (c->device >= 0) HIPCHK(c, hipSetDevice(c->device));
    if (c->device >= 0) HIPCHK(c, hipDeviceSynchronize());
    c->drop_apply_graph();
    c->graphs = enable != 0;
    return CHI0_OK;
}

// chi0_apply without allocation: every workspace buffer of the operator is
// carved from the device's static scratch (offsets in doubles, 256-byte
// aligned); no split-K partials beyond what fits, no tile tuning, no timing.
namespace {
struct ScratchLayout {
    int64_t omega, Zin, Yout, dV, W, Tt, Ut, at, part, gemm, end;
};
ScratchLayout scratch_layout(const chi0_ctx *c, int nb) {
    const int64_t nc = 2 * nb, mcol = (int64_t)c->No_pad * nc;
    ScratchLayout L{};
    int64_t o = 0;
    auto take = [&](int64_t n) { const int64_t at = o; o += round_up(std::max<int64_t>(n, 1), 32); return at; };
    L.omega = take(nb);
    L.Zin = take((int64_t)c->P_pad * nc);
    L.Yout = take((int64_t)c->P_pad * nc);
    L.dV = take(c->nnzB * nc);
    L.W = take(c->nnzB * nc);
    L.Tt = take((int64_t)c->N_pad * mcol);
    L.Ut = take((int64_t)c->N_pad * mcol);
    L.at = take((int64_t)c->Nv_pad * mcol);
    L.part = take(c->npart * nc);
    L.gemm = o;   // split-K partials: whatever is left (none if too little)
    L.end = o;
    return L;
}
}  // namespace

extern "C" int chi0_apply_noalloc(chi0_ctx *c, int32_t n_rhs, const double *omega, double eps,
                                  const double *z, double *out, void *stream) {
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    if (n_rhs < 0) return fail(c, CHI0_EINVAL, "n_rhs < 0");
    if (n_rhs == 0) return CHI0_OK;
    if (!omega || !z || !out) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (!all_finite(omega, n_rhs)) return fail(c, CHI0_ENONFINITE, "non-finite omega");
    if (n_rhs > kMaxBatch) return fail(c, CHI0_EINVAL, "n_rhs must be <= 256");
    const ScratchLayout L = scratch_layout(c, n_rhs);
    if (L.end > kScratchDoubles) {
        int fit = 0;
        while (fit < kMaxBatch && scratch_layout(c, fit + 1).end <= kScratchDoubles) ++fit;
        return fail(c, CHI0_EINVAL, "chi0_apply_noalloc: " + std::to_string(n_rhs) + " right-hand sides need " +
                                        std::to_string(L.end * 8) + " bytes of workspace, the static scratch holds " +
                                        std::to_string(kScratchDoubles * 8) + "; at most " + std::to_string(fit) +
                                        " fit for this system (chi0_apply has no such limit)");
    }
    double *base = c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
    if (!base) return fail(c, CHI0_EHIP, "static scratch address not set up for this device");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    OpWork o;   // a view into the scratch: owns nothing
    o.omega_dev = base + L.omega;
    o.Zin = base + L.Zin;
    o.Yout = base + L.Yout;
    o.dV = base + L.dV;
    o.W = base + L.W;
    o.Tt = base + L.Tt;
    o.Ut = base + L.Ut;
    o.at = base + L.at;
    o.part = base + L.part;
    const int64_t left = kScratchDoubles - L.gemm;
    o.gemm_scratch = left >= 2 * 64 * 64 ? base + L.gemm : nullptr;
    o.gemm_scratch_n = o.gemm_scratch ? (size_t)left : 0;
    const int nc = 2 * n_rhs;
    // The scratch keeps the last call's contents (any system, any n_rhs): clear
    // the buffers this call uses, whose padding the GEMMs read as zeros.
    launch_zero(nullptr, s, base, L.gemm);
    HIPCHK(c, hipMemcpyAsync(o.omega_dev, omega, (size_t)n_rhs * 8, hipMemcpyHostToDevice, s));
    launch_rows_to_cols(nullptr, s, z, n_rhs, c->P, o.Zin, nc);
    run_chi0(c, o, s, n_rhs, eps, CHI0_PREC_FP64, o.omega_dev, nullptr, nullptr);
    launch_cols_to_rows(nullptr, s, o.Yout, n_rhs, c->P, nc, out);
    HIPCHK(c, hipGetLastError());
    return CHI0_OK;
}

// ================================================================== solver
static int ensure_slots(chi0_ctx *c, int n, int m) {
    if (n <= c->slot_n && m == c->slot_m) return CHI0_OK;
    for (hipStream_t ls : c->lane_stream)
        if (ls) HIPCHK(c, hipStreamSynchronize(ls));
    c->slotbuf.release();
    c->slot_n = c->slot_m = 0;
    DevBuf &b = c->slotbuf;
    SlotsDev &sl = c->slots;
    sl.m = m;
    sl.P_pad = c->P_pad;
    sl.vstride = (int64_t)(m + 1) * c->P_pad * 2;
    sl.hstride = (int64_t)m * (m + 3) / 2 * 2;
    sl.hbstride = (int64_t)(3 * m + 4) * 2;
    CHK(dalloc(c, b, &sl.V, n * sl.vstride));
    CHK(dalloc(c, b, &sl.H, n * sl.hstride));
    CHK(dalloc(c, b, &sl.cs, (int64_t)n * m));
    CHK(dalloc(c, b, &sl.sn, (int64_t)n * m * 2));
    CHK(dalloc(c, b, &sl.g, (int64_t)n * (m + 1) * 2));
    CHK(dalloc(c, b, &sl.x, (int64_t)n * c->P_pad * 2));
    CHK(dalloc(c, b, &sl.b, (int64_t)n * c->P_pad * 2));
    CHK(dalloc(c, b, &sl.hbuf, (int64_t)n * sl.hbstride));
    CHK(dalloc(c, b, &sl.y, (int64_t)n * m * 2));
    CHK(dalloc(c, b, &sl.w, (int64_t)n * c->P_pad * 2));
    const int64_t ab = (int64_t)n * (sizeof(Job) + sizeof(double));
    double *arena = nullptr;
    CHK(dalloc(c, b, &arena, kSets * ab / 8));
    c->arena_dev = reinterpret_cast<char *>(arena);
    CHK(dalloc(c, b, &c->fin_dev, kSets * n));
    CHK(dalloc(c, b, &c->upd_dev, kSets * n));
    CHK(dalloc(c, b, &c->status_dev, kSets * n));
    if (c->host_cap != n) {   // the host arena's layout depends on n
        if (c->arena_h) (void)hipHostFree(c->arena_h);
        if (c->fin_h) (void)hipHostFree(c->fin_h);
        if (c->upd_h) (void)hipHostFree(c->upd_h);
        if (c->status_h) (void)hipHostFree(c->status_h);
        c->arena_h = nullptr;
        c->fin_h = c->upd_h = nullptr;
        c->status_h = nullptr;
        c->host_cap = 0;
        HIPCHK(c, hipHostMalloc((void **)&c->arena_h, kSets * ab, hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void **)&c->fin_h, sizeof(Job) * kSets * n, hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void **)&c->upd_h, sizeof(Job) * kSets * n, hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void **)&c->status_h, sizeof(StepStatus) * kSets * n, hipHostMallocDefault));
        c->host_cap = n;
    }
    for (hipEvent_t &e : c->step_ev)
        if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(c, hipDeviceSynchronize());
    c->slot_n = n;
    c->slot_m = m;
    return CHI0_OK;
}

namespace {
enum { S_FREE = 0, S_RHS, S_ARNOLDI, S_RESID };
struct SlotState {
    int state = S_FREE;
    int point = -1;
    int j = 0;                   // next Arnoldi index to launch in the current cycle
    int pend = 0;                // launched Arnoldi steps of this cycle not yet seen by the host
    int epoch = 0;               // bumped when a cycle ends: steps launched before are void
    bool busy = false;           // a b or residual job of this slot is in flight
    int prec = CHI0_PREC_FP64;   // arithmetic of this slot's Arnoldi steps
    bool warm_check = false;     // the pending residual job checks a warm start
    double bnorm = 0.0;          // ||b|| = ||chi0 d||
    double cycle0 = 0.0;         // residual norm at the start of the current cycle
    double rel_prev = 1.0;       // true relative residual after the previous cycle
    bool eps_met = false;        // the cycle ended by the eps_P / eps_X test
};
struct PointState {
    int iters = 0, restarts = 0, converged = 0, breakdown = 0, fallback = 0, warm = 0, low = 0;
    double rel = NAN, warm_rel0 = 0.0, eps_x = 0.0, eps_p = 0.0;
};
}  // namespace

// ============================================================ warm start
struct chi0_ws {
    chi0_ctx *ctx = nullptr;
    int r = 0;            // basis size
    int F = 0;            // input features (2 n_freq)
    int W = 0;            // hidden width
    int O = 0;            // network outputs (2 r rounded up to 32)
    int nf = 0;
    double w_scale = 1.0;
    int epochs = 0;
    DevBuf buf;
    double *U = nullptr;  // [r][P_pad] complex
    float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
    int64_t n_params = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    float *mean = nullptr, *sdev = nullptr;   // [O] output de-normalisation
    // activations for batches of up to kMaxBatch rows
    float *phi = nullptr, *H1 = nullptr, *H2 = nullptr, *out = nullptr, *dout = nullptr, *dH1 = nullptr,
          *dH2 = nullptr, *tgt = nullptr, *loss = nullptr;
    double *omega_dev = nullptr;
    Job *jobs_dev = nullptr;
    std::vector<float> loss_hist;
    ~chi0_ws() { buf.release(); }
};

namespace {
// Forward pass for `rows` (multiple of 32) feature rows already in ws->phi.
void ws_forward(chi0_ws *w, hipStream_t s, int rows) {
    float *P = w->params;
    launch_mlp_gemm(s, rows, w->W, w->F, w->phi, w->F, 1, P + w->oW1, 1, w->F, w->H1, w->W);
    launch_bias_act(s, rows, w->W, w->H1, P + w->ob1, 1);
    launch_mlp_gemm(s, rows, w->W, w->W, w->H1, w->W, 1, P + w->oW2, 1, w->W, w->H2, w->W);
    launch_bias_act(s, rows, w->W, w->H2, P + w->ob2, 1);
    launch_mlp_gemm(s, rows, w->O, w->W, w->H2, w->W, 1, P + w->oW3, 1, w->W, w->out, w->O);
    launch_bias_act(s, rows, w->O, w->out, P + w->ob3, 0);
}

// Loss of rows [0, n_rows) against ws->tgt and all parameter gradients into ws->grads.
void ws_backward(chi0_ws *w, hipStream_t s, int rows, int n_rows, int n_cols, float *loss) {
    float *P = w->params, *G = w->grads;
    launch_mse(s, rows, w->O, n_rows, n_cols, w->out, w->tgt, w->dout, loss);
    launch_mlp_gemm(s, w->O, w->W, rows, w->dout, 1, w->O, w->H2, w->W, 1, G + w->oW3, w->W);
    launch_colsum(s, rows, w->O, w->dout, G + w->ob3);
    launch_mlp_gemm(s, rows, w->W, w->O, w->dout, w->O, 1, P + w->oW3, w->W, 1, w->dH2, w->W);
    launch_tanh_back(s, (int64_t)rows * w->W, w->H2, w->dH2);
    launch_mlp_gemm(s, w->W, w->W, rows, w->dH2, 1, w->W, w->H1, w->W, 1, G + w->oW2, w->W);
    launch_colsum(s, rows, w->W, w->dH2, G + w->ob2);
    launch_mlp_gemm(s, rows, w->W, w->W, w->dH2, w->W, 1, P + w->oW2, w->W, 1, w->dH1, w->W);
    launch_tanh_back(s, (int64_t)rows * w->W, w->H1, w->dH1);
    launch_mlp_gemm(s, w->W, w->F, rows, w->dH1, 1, w->W, w->phi, w->F, 1, G + w->oW1, w->F);
    launch_colsum(s, rows, w->W, w->dH1, G + w->ob1);
}

// Network forward for n frequencies (host array) -> ws->out rows [0, n).
int ws_infer(chi0_ws *w, hipStream_t s, int n, const double *omega_host) {
    chi0_ctx *c = w->ctx;
    const int rows = (int)round_up(std::max(n, 1), 32);
    HIPCHK(c, hipMemcpyAsync(w->omega_dev, omega_host, sizeof(double) * n, hipMemcpyHostToDevice, s));
    launch_features(s, n, rows, w->omega_dev, w->nf, w->w_scale, w->phi);
    ws_forward(w, s, rows);
    return CHI0_OK;
}
}  // namespace

// ================================================================= solver
// x_out: optional DEVICE [npts][P_pad] complex, the solution of each point.
static int solve_impl(chi0_ctx *c, int32_t n_omega, const double *omega, double eps, int32_t n_drive,
                      const double *V_ext, const chi0_solve_opts *opts_in, double *alpha,
                      chi0_point_stats *stats, double *x_out) {
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    chi0_solve_opts o;
    chi0_solve_opts_default(&o);
    if (opts_in) o = *opts_in;
    if (n_omega < 0 || n_drive < 1 || n_drive > 3) return fail(c, CHI0_EINVAL, "need n_omega >= 0, 1 <= n_drive <= 3");
    if (n_omega == 0) return CHI0_OK;
    if (!omega || !V_ext || !alpha) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (o.restart < 1 || o.restart > 32767) return fail(c, CHI0_EINVAL, "restart must be in [1, 32767]");
    if (o.max_iter < 1) return fail(c, CHI0_EINVAL, "max_iter must be >= 1");
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(c, CHI0_EINVAL, "tol must be finite and > 0");
    if (o.batch < 1) return fail(c, CHI0_EINVAL, "batch must be >= 1");
    if (o.batch > kMaxBatch) return fail(c, CHI0_EINVAL, "batch must be <= 256");
    if (o.precision < CHI0_PREC_FP64 || o.precision > CHI0_PREC_BF16X3)
        return fail(c, CHI0_EINVAL, "unknown precision");
    if (!(o.inner_tol >= 0.0) || !(o.inner_tol < 1.0)) return fail(c, CHI0_EINVAL, "inner_tol must be in [0, 1)");
    if (o.mixed != CHI0_MIXED_REFINE && o.mixed != CHI0_MIXED_RELAXED) return fail(c, CHI0_EINVAL, "unknown mixed");
    if (!(o.relax >= 0.0) || !std::isfinite(o.relax)) return fail(c, CHI0_EINVAL, "relax must be finite and >= 0");
    if (o.alpha_form != CHI0_ALPHA_CORRECTED && o.alpha_form != CHI0_ALPHA_PLAIN)
        return fail(c, CHI0_EINVAL, "unknown alpha_form");
    if (o.stop < CHI0_STOP_RESIDUAL || o.stop > CHI0_STOP_EPS_PX) return fail(c, CHI0_EINVAL, "unknown stop");
    if (o.lanes < 0 || o.lanes > kLanes) return fail(c, CHI0_EINVAL, "lanes must be 0 (auto) or 1..4");
    if (o.ortho < CHI0_ORTHO_AUTO || o.ortho > CHI0_ORTHO_DCGS2) return fail(c, CHI0_EINVAL, "unknown ortho");
    // delayed reorthogonalisation needs a few columns per cycle (one is always provisional)
    const bool dcgs = o.ortho == CHI0_ORTHO_DCGS2 || (o.ortho == CHI0_ORTHO_AUTO && o.restart >= 8);
    if (dcgs && o.restart < 3) return fail(c, CHI0_EINVAL, "DCGS2 needs restart >= 3");
    // CGS2 stages a step's coefficients in LDS (64 KB: 4095 complex)
    if (!dcgs && o.restart > 4095) return fail(c, CHI0_EINVAL, "CGS2 needs restart <= 4095");
    const bool use_eps = o.stop != CHI0_STOP_RESIDUAL;
    if (use_eps && (!dcgs || o.precision != CHI0_PREC_FP64))
        return fail(c, CHI0_EINVAL, "the eps_P / eps_X stopping tests need DCGS2 steps in FP64");
    // learned warm start of each drive: `warm` for all of them, or one per drive
    if (o.warm && o.warm_drive) return fail(c, CHI0_EINVAL, "warm and warm_drive are exclusive");
    std::vector<chi0_ws *> wsd(n_drive, nullptr);
    for (int i = 0; i < n_drive; ++i) {
        wsd[i] = const_cast<chi0_ws *>(o.warm_drive ? o.warm_drive[i] : o.warm);
        if (wsd[i] && wsd[i]->ctx != c) return fail(c, CHI0_EINVAL, "warm start belongs to another context");
    }
    const bool any_ws = std::any_of(wsd.begin(), wsd.end(), [](chi0_ws *w) { return w != nullptr; });
    const double *x0 = o.x0;
    if (any_ws && x0) return fail(c, CHI0_EINVAL, "a learned warm start and x0 are exclusive");
    // whether point p starts from a given vector (x0 or its drive's network) rather than 0
    auto started = [&](int p) { return x0 != nullptr || wsd[p % n_drive] != nullptr; };
    const double inner_tol = o.inner_tol > 0.0 ? o.inner_tol
                             : (o.precision == CHI0_PREC_FP32 ? 1e-6 : 1e-4);
    // relaxed low precision: a point's Arnoldi steps leave FP64 once the
    // residual estimate is at most relax_at ||b|| (the operator error allowed
    // by tol ||b|| / ||r|| has then grown to the low-precision operator's own)
    const bool relaxed = o.precision != CHI0_PREC_FP64 && o.mixed == CHI0_MIXED_RELAXED;
    const double relax_at = (o.relax > 0.0 ? o.relax : 1.0) * o.tol /
                            (o.precision == CHI0_PREC_FP32 ? kOpErrFP32 : kOpErrBF16X3);
    if (!all_finite(omega, n_omega)) return fail(c, CHI0_ENONFINITE, "non-finite omega");
    if (!all_finite(V_ext, (int64_t)n_drive * c->P)) return fail(c, CHI0_ENONFINITE, "non-finite V_ext");
    HIPCHK(c, hipSetDevice(c->device));

    const int npts = n_omega * n_drive;
    // storage for m columns per cycle; the delayed scheme keeps one extra
    // provisional column, so it gets one more basis vector
    const int m = o.restart + (dcgs ? 1 : 0);
    const int P = c->P;
    // per-call device buffers: drives, alpha, and the residuals r and adjoint
    // vectors d + K x of every point for the cross-drive residual terms
    DevBuf callbuf;
    // on every exit (also an error with steps in flight) drain the lanes first
    struct Guard {
        DevBuf *b;
        chi0_ctx *c;
        ~Guard() {
            for (hipStream_t ls : c->lane_stream)
                if (ls) (void)hipStreamSynchronize(ls);
            b->release();
        }
    } guard{&callbuf, c};
    const bool correct = o.alpha_form == CHI0_ALPHA_CORRECTED;
    double *Rst = nullptr, *Wst = nullptr;
    if (correct && n_drive > 1) {
        CHK(dalloc(c, callbuf, &Rst, (int64_t)npts * P * 2));
        CHK(dalloc(c, callbuf, &Wst, (int64_t)npts * P * 2));
    }
    // Concurrent slots: the batch, capped so that the slots' Krylov bases and
    // Hessenberg matrices (and R^-1 of the error estimates) fit in the device
    // memory that is free, less a reserve for the operator workspaces.
    int nsl = std::min(std::min(o.batch, npts), kMaxBatch);
    if (!(c->slot_n >= nsl && c->slot_m == m)) {
        const double per_slot = 8.0 * (2.0 * (m + 1) * c->P_pad + (double)m * (m + 3) + 6.0 * c->P_pad +
                                       16.0 * m + 16.0) +
                                (o.stop != CHI0_STOP_RESIDUAL ? 8.0 * ((double)m * (m + 1) + 8.0 * m + 16.0) : 0.0);
        size_t free_b = 0, total_b = 0;
        HIPCHK(c, hipMemGetInfo(&free_b, &total_b));
        const double held = (double)c->slot_n * (c->slot_m > 0 ? 8.0 * (2.0 * (c->slot_m + 1) * c->P_pad +
                                                                        (double)c->slot_m * (c->slot_m + 3)) : 0.0);
        const double avail = (double)free_b + held - 0.05 * (double)total_b - 4e9;
        const int fit = avail > per_slot ? (int)std::min(avail / per_slot, 1e6) : 1;
        nsl = std::max(1, std::min(nsl, fit));
    }
    // Slots are dealt to lanes (slot k to lane k mod nl), each lane with its own
    // stream, operator workspace and step buffers, so that one lane's
    // memory-bound Gram-Schmidt passes can run beside the other lane's
    // matrix-core transforms.  Dealing the slots mixes the frequencies, whose
    // iteration counts differ by up to 5x, over both lanes.  Small batches use
    // one lane.
    const int nl = std::min(nsl, o.lanes > 0 ? o.lanes : (nsl >= 16 ? kAutoLanes : 1));
    for (int L = 0; L < nl; ++L) {
        const int ln = (nsl - L + nl - 1) / nl;
        CHK(ensure_ws(c, c->op[L], 2 * std::max(ln, c->op[L].nc_cap / 2)));
        if (o.precision != CHI0_PREC_FP64) CHK(ensure_lp(c, c->op[L]));
    }
    CHK(ensure_slots(c, nsl, m));
    Tracer *t = &c->tracer;

    double *drives = nullptr, *alpha_dev = nullptr;
    CHK(dalloc(c, callbuf, &drives, (int64_t)n_drive * c->P_pad));
    CHK(dalloc(c, callbuf, &alpha_dev, (int64_t)npts * n_drive * 2));
    HIPCHK(c, hipMemcpy2D(drives, (size_t)c->P_pad * 8, V_ext, (size_t)P * 8, (size_t)P * 8,
                          (size_t)n_drive, hipMemcpyHostToDevice));
    // error estimates of the paper's stopping test: R^-1, y, d.v_i, x0^H v_i per slot
    EpsDev epsd{};
    if (use_eps) {
        epsd.zstride = (int64_t)m * (m + 1);   // m(m+1)/2 complex
        CHK(dalloc(c, callbuf, &epsd.Z, nsl * epsd.zstride));
        CHK(dalloc(c, callbuf, &epsd.yv, (int64_t)nsl * m * 2));
        CHK(dalloc(c, callbuf, &epsd.dl, (int64_t)nsl * (m + 1) * 2));
        CHK(dalloc(c, callbuf, &epsd.xi, (int64_t)nsl * (m + 1) * 2));
        CHK(dalloc(c, callbuf, &epsd.st, (int64_t)nsl * EPS_NS));
        epsd.drives = drives;
    }
    HIPCHK(c, hipDeviceSynchronize());

    std::vector<SlotState> sl(nsl);
    std::vector<PointState> ps(npts);
    int next_point = 0, done = 0;

    // Each lane keeps two steps in flight.  While the GPU runs step s+1 the
    // host reads the status of step s and decides what step s+2 does.  A slot
    // in its Arnoldi phase is launched again before the host has seen its
    // previous step; if that previous step ends the cycle, the extra step is
    // void (its epoch no longer matches).  It only wrote basis vectors,
    // Hessenberg columns and rotations beyond the cycle's length L, which the
    // update of x never reads.  b and residual jobs are never launched ahead.
    struct InFlight {
        int nb = 0, nb64 = 0;   // jobs [nb64, nb) are reduced-precision Arnoldi steps
        int64_t seq = 0;
        std::vector<int> epoch;
    } fl[kSets];
    struct LaneState {
        int q_launch = 0, n_inflight = 0, q_oldest = 0, last_q = 0;
        std::vector<Job> fin, upd, rst, wnew, xnew;
        std::vector<double> wom;
    } lanes[kLanes];
    for (int L = 0; L < nl; ++L) lanes[L].q_launch = lanes[L].q_oldest = lanes[L].last_q = 2 * L;
    int64_t seq = 0;

    auto plan_and_launch = [&](int L, int q) -> int {
        hipStream_t s = c->lane_stream[L];
        OpWork &ow = c->op[L];
        Job *jobs_h = c->jobs_h(q);
        double *om_h = c->omega_h(q);
        InFlight &f = fl[q];
        f.epoch.clear();
        int nb = 0, nb64 = 0, jmax = -1, n_arn = 0;
        double sum_j1 = 0.0;
        // FP64 jobs first (b, true residual, FP64 Arnoldi), then the
        // low-precision Arnoldi steps: each group is one operator pass
        for (int pass = 0; pass < 2; ++pass)
            for (int k = L; k < nsl; k += nl) {
                SlotState &ss = sl[k];
                if (ss.state == S_FREE || ss.busy) continue;
                const bool lowp = ss.state == S_ARNOLDI && ss.prec != CHI0_PREC_FP64;
                if (lowp != (pass == 1)) continue;
                Job jb;
                jb.slot = k;
                jb.drive = ss.point % n_drive;
                if (ss.state == S_ARNOLDI) {
                    if (ss.j >= m || ps[ss.point].iters + ss.pend >= o.max_iter) continue;
                    jb.type = JOB_ARNOLDI;
                    jb.j = ss.j++;
                    ss.pend += 1;
                    jmax = std::max(jmax, jb.j);
                    ++n_arn;
                    sum_j1 += jb.j + 1;
                } else {
                    jb.type = ss.state == S_RHS ? JOB_RHS : JOB_RESID;
                    jb.j = jb.type == JOB_RHS ? (started(ss.point) ? 1 : 0) : 0;
                    ss.busy = true;
                }
                jobs_h[nb] = jb;
                om_h[nb] = omega[ss.point / n_drive];
                f.epoch.push_back(ss.epoch);
                ++nb;
                if (pass == 0) ++nb64;
            }
        f.nb = nb;
        f.nb64 = nb64;
        f.seq = seq++;
        if (nb == 0) return CHI0_OK;
        Job *jobs_d = c->jobs_dev(q);
        double *om_d = c->somega_dev(q);
        StepStatus *st_d = c->status_dev + q * nsl;
        HIPCHK(c, hipMemcpyAsync(jobs_d, jobs_h, c->slot_n * sizeof(Job) + nb * sizeof(double),
                                 hipMemcpyHostToDevice, s));
        // operator per group: Zin = K v (b jobs: d), Y = chi0 Zin, then post
        auto run_group = [&](int g0, int gn, int prec) {
            const int nc = 2 * gn;
            const Job *jg = jobs_d + g0;
            launch_gather_jobs(t, s, jg, gn, c->slots, ow.Vb, nc, P);
            if (nc <= 32)
                launch_kmatvec_skinny(t, s, c->P_pad, c->K, ow.Vb, ow.Zin, nc, (double)P);
            else
                launch_dgemm(t, s, "kernel_matmul", c->P_pad, nc, c->P_pad, c->P_pad, c->K, c->P_pad, ow.Vb, nc, ow.Zin,
                             nc, 2.0 * P * (double)P * nc, 8.0 * ((double)P * P + 2.0 * P * nc),
                             ow.gemm_scratch, ow.gemm_scratch_n, &c->tuner);
            launch_put_drive(t, s, jg, gn, drives, c->P_pad, ow.Zin, nc, P);
            run_chi0(c, ow, s, gn, eps, prec, om_d + g0, t, &c->tuner);
            launch_post_jobs(t, s, jg, gn, c->slots, ow.Yout, ow.Zin, drives, nc, P, st_d + g0);
        };
        if (nb64 > 0) run_group(0, nb64, CHI0_PREC_FP64);
        if (nb > nb64) run_group(nb64, nb - nb64, o.precision);
        if (n_arn > 0) {
            if (dcgs)
                launch_dcgs(t, s, jobs_d, nb, jmax, c->slots, P, st_d, n_arn, sum_j1, ow.gemm_scratch,
                            ow.gemm_scratch_n, use_eps ? &epsd : nullptr);
            else
                launch_arnoldi(t, s, jobs_d, nb, jmax, c->slots, P, st_d, n_arn, sum_j1);
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->status_h + q * nsl, st_d, sizeof(StepStatus) * nb, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipEventRecord(c->step_ev[q], s));
        return CHI0_OK;
    };

    // relaxed low precision: the arithmetic a cycle starts in, from its residual norm
    auto start_prec = [&](double rnorm, double bnorm) {
        return rnorm <= relax_at * bnorm ? o.precision : (int32_t)CHI0_PREC_FP64;
    };

    // Advance the slot state machines of lane L with the status of its step in set q.
    auto process = [&](int L, int q) {
        LaneState &ln = lanes[L];
        const InFlight &f = fl[q];
        const Job *jobs_h = c->jobs_h(q);
        const StepStatus *sts = c->status_h + q * nsl;
        for (int r = 0; r < f.nb; ++r) {
            const Job &jb = jobs_h[r];
            SlotState &ss = sl[jb.slot];
            const StepStatus &st = sts[r];
            if (jb.type == JOB_ARNOLDI) {
                if (f.epoch[r] != ss.epoch || ss.state != S_ARNOLDI) continue;   // void step
                PointState &pt = ps[ss.point];
                ss.pend -= 1;
                pt.iters += 1;
                if (r >= f.nb64) pt.low += 1;
                double stop = o.tol * ss.bnorm;
                if (relaxed) {
                    if (ss.prec == CHI0_PREC_FP64 && !pt.fallback && st.value <= relax_at * ss.bnorm)
                        ss.prec = o.precision;   // for the steps launched from now on
                } else if (ss.prec != CHI0_PREC_FP64) {
                    stop = std::max(stop, inner_tol * ss.cycle0);
                }
                const bool brk = st.hnext == 0.0;
                if (brk) pt.breakdown = 1;
                // CGS2: the step completes column j (dimension j+1).  Delayed
                // reorthogonalisation: it completes column j-1 (dimension j) and
                // leaves column j provisional, so a cycle uses the first j columns.
                const int Lc = dcgs ? jb.j : jb.j + 1;
                bool crit = st.value <= stop;
                if (use_eps) {   // Sec. 4.1: eps_P alone, or eps_P and eps_X
                    pt.eps_x = st.eps_x;
                    pt.eps_p = st.eps_p;
                    crit = st.eps_p <= o.tol && (o.stop != CHI0_STOP_EPS_PX || st.eps_x <= o.tol);
                }
                const bool est_ok = Lc >= 1 && crit;
                if (est_ok || brk || jb.j + 1 >= m || pt.iters >= o.max_iter || !std::isfinite(st.value)) {
                    if (Lc >= 1) ln.upd.push_back({jb.slot, 0, Lc, 0});
                    ss.state = S_RESID;
                    ss.epoch += 1;
                    ss.pend = 0;
                    ss.eps_met = use_eps && est_ok;
                }
                continue;
            }
            PointState &pt = ps[ss.point];
            ss.busy = false;
            if (jb.type == JOB_RHS) {
                ss.bnorm = st.value;
                ss.cycle0 = st.value;
                ss.rel_prev = 1.0;
                ss.prec = relaxed ? start_prec(ss.cycle0, ss.bnorm) : o.precision;
                if (!(st.value > 0.0) || !std::isfinite(st.value)) {
                    pt.rel = st.value == 0.0 ? 0.0 : NAN;
                    pt.converged = st.value == 0.0;
                    if (started(ss.point)) ln.rst.push_back({jb.slot, 0, 0, 0});   // x = 0 is the answer
                    ln.fin.push_back({jb.slot, 0, ss.point, 0});
                    ss.state = S_FREE;
                    ++done;
                } else if (started(ss.point)) {
                    ss.state = S_RESID;       // r0 = b - A x0 decides on the warm start
                    ss.warm_check = true;
                } else {
                    ss.state = S_ARNOLDI;
                    ss.j = 0;
                    ss.pend = 0;
                }
            } else if (ss.warm_check) {
                ss.warm_check = false;
                const double rel0 = st.value / ss.bnorm;
                pt.rel = rel0;
                pt.warm_rel0 = rel0;
                if (rel0 <= o.tol) {                        // the warm start is already the answer
                    pt.warm = 1;
                    pt.converged = 1;
                    ln.fin.push_back({jb.slot, 0, ss.point, 0});
                    ss.state = S_FREE;
                    ++done;
                } else if (!(rel0 < 1.0)) {                 // no better than x0 = 0: zero start
                    pt.warm = 2;
                    ln.rst.push_back({jb.slot, 0, 0, 0});
                    ss.cycle0 = ss.bnorm;
                    ss.rel_prev = 1.0;
                    ss.state = S_ARNOLDI;
                    ss.j = 0;
                    ss.pend = 0;
                } else {
                    pt.warm = 1;
                    ss.cycle0 = st.value;
                    ss.rel_prev = rel0;
                    if (relaxed) ss.prec = start_prec(ss.cycle0, ss.bnorm);
                    ss.state = S_ARNOLDI;
                    ss.j = 0;
                    ss.pend = 0;
                }
            } else {
                pt.restarts += 1;
                pt.rel = st.value / ss.bnorm;
                if (pt.rel <= o.tol || ss.eps_met || pt.iters >= o.max_iter || !std::isfinite(pt.rel)) {
                    pt.converged = pt.rel <= o.tol || ss.eps_met;
                    ln.fin.push_back({jb.slot, 0, ss.point, 0});
                    ss.state = S_FREE;
                    ++done;
                } else {
                    // iterative refinement: a low-precision cycle that did not halve the
                    // true residual hands the point to FP64 Arnoldi steps
                    if (ss.prec != CHI0_PREC_FP64 && pt.rel > 0.5 * ss.rel_prev) {
                        ss.prec = CHI0_PREC_FP64;
                        pt.fallback = 1;
                    } else if (relaxed && !pt.fallback) {   // by the residual the new cycle starts from
                        ss.prec = start_prec(st.value, ss.bnorm);
                    }
                    ss.rel_prev = pt.rel;
                    ss.cycle0 = st.value;
                    ss.state = S_ARNOLDI;
                    ss.j = 0;
                    ss.pend = 0;
                }
            }
        }
    };

    // Work of lane L decided by its last processed status, issued on its
    // stream before its next step.  Each list uses the host set q of that
    // status's step: the set is rewritten only after the host has waited for
    // the set's next step, which follows these copies on the stream.
    auto issue_pending = [&](int L, int q) -> int {
        LaneState &ln = lanes[L];
        hipStream_t s = c->lane_stream[L];
        Job *fin_h = c->fin_h + q * nsl, *upd_h = c->upd_h + q * nsl;
        Job *fin_d = c->fin_dev + q * nsl, *upd_d = c->upd_dev + q * nsl;
        if (!ln.rst.empty()) {   // zero start for rejected warm starts (and x = 0 where b = 0)
            HIPCHK(c, hipStreamSynchronize(s));   // upd_h is reused below
            std::copy(ln.rst.begin(), ln.rst.end(), upd_h);
            HIPCHK(c, hipMemcpyAsync(upd_d, upd_h, sizeof(Job) * ln.rst.size(), hipMemcpyHostToDevice, s));
            launch_reset_slots(s, upd_d, (int)ln.rst.size(), c->slots, P);
            HIPCHK(c, hipStreamSynchronize(s));
            ln.rst.clear();
        }
        // polarizability (and stored solution) of finished points, before the slot is reused
        if (!ln.fin.empty()) {
            std::copy(ln.fin.begin(), ln.fin.end(), fin_h);
            HIPCHK(c, hipMemcpyAsync(fin_d, fin_h, sizeof(Job) * ln.fin.size(), hipMemcpyHostToDevice, s));
            launch_alpha(t, s, fin_d, (int)ln.fin.size(), c->slots, drives, n_drive, c->P_pad, P, correct,
                         Rst, Wst, alpha_dev);
            if (x_out) launch_store_x(s, fin_d, (int)ln.fin.size(), c->slots, P, x_out);
            ln.fin.clear();
        }
        // x += V y for slots that ended a cycle
        if (!ln.upd.empty()) {
            int jm = 0;
            double sumL = 0.0;
            for (auto &u : ln.upd) {
                jm = std::max(jm, u.j);
                sumL += u.j;
            }
            std::copy(ln.upd.begin(), ln.upd.end(), upd_h);
            HIPCHK(c, hipMemcpyAsync(upd_d, upd_h, sizeof(Job) * ln.upd.size(), hipMemcpyHostToDevice, s));
            launch_update_x(t, s, upd_d, (int)ln.upd.size(), jm, c->slots, P, sumL);
            ln.upd.clear();
        }
        // points new in this lane's slots with a given start vector get it now
        for (const Job &jn : ln.xnew)
            HIPCHK(c, hipMemcpyAsync(c->slots.x + (int64_t)jn.slot * c->P_pad * 2, x0 + (int64_t)jn.j * P * 2,
                                     (size_t)P * 16, hipMemcpyDeviceToDevice, s));
        ln.xnew.clear();
        // warm-started points new in this lane's slots get x0 = U c(omega) now,
        // from the network of their drive (one inference per network)
        if (!ln.wnew.empty()) {
            std::vector<Job> grp;
            std::vector<double> gom;
            for (int d = 0; d < n_drive; ++d) {
                chi0_ws *ws = wsd[d];
                grp.clear();
                gom.clear();
                for (size_t q = 0; q < ln.wnew.size(); ++q)
                    if (ln.wnew[q].drive == d) {
                        grp.push_back(ln.wnew[q]);
                        gom.push_back(ln.wom[q]);
                    }
                if (grp.empty() || !ws) continue;
                // the network's buffers are shared by the lanes: this stream finishes
                // its inference before the host moves on (and fin_h is reused)
                HIPCHK(c, hipStreamSynchronize(s));
                std::copy(grp.begin(), grp.end(), fin_h);
                HIPCHK(c, hipMemcpyAsync(ws->jobs_dev, fin_h, sizeof(Job) * grp.size(), hipMemcpyHostToDevice, s));
                CHK(ws_infer(ws, s, (int)grp.size(), gom.data()));
                launch_ws_apply(s, ws->jobs_dev, (int)grp.size(), ws->out, ws->O, ws->mean, ws->sdev, ws->r,
                                ws->U, (int64_t)c->P_pad * 2, c->slots.x, (int64_t)c->P_pad * 2, P);
                HIPCHK(c, hipStreamSynchronize(s));
            }
            ln.wnew.clear();
            ln.wom.clear();
        }
        return CHI0_OK;
    };

    // Free slots take the next points in slot order, so consecutive points
    // (neighbouring frequencies, alike in cost) alternate between the lanes.
    auto refill = [&]() {
        for (int k = 0; k < nsl; ++k)
            if (sl[k].state == S_FREE && !sl[k].busy && next_point < npts) {
                sl[k].state = S_RHS;
                sl[k].point = next_point++;
                sl[k].j = 0;
                sl[k].pend = 0;
                sl[k].epoch += 1;
                sl[k].warm_check = false;
                sl[k].eps_met = false;
                if (wsd[sl[k].point % n_drive]) {
                    LaneState &ln = lanes[k % nl];
                    ln.wnew.push_back({k, 0, sl[k].point, sl[k].point % n_drive});
                    ln.wom.push_back(omega[sl[k].point / n_drive]);
                } else if (x0) {
                    lanes[k % nl].xnew.push_back({k, 0, sl[k].point, 0});
                }
            }
    };

    for (;;) {
        refill();
        for (int L = 0; L < nl; ++L) {
            LaneState &ln = lanes[L];
            CHK(issue_pending(L, ln.last_q));
            while (ln.n_inflight < 2) {
                CHK(plan_and_launch(L, ln.q_launch));
                if (fl[ln.q_launch].nb == 0) break;
                if (ln.n_inflight == 0) ln.q_oldest = ln.q_launch;
                ++ln.n_inflight;
                ln.q_launch ^= 1;   // sets 2L and 2L+1
            }
        }
        // process the oldest step over all lanes
        int Lw = -1;
        for (int L = 0; L < nl; ++L)
            if (lanes[L].n_inflight > 0 && (Lw < 0 || fl[lanes[L].q_oldest].seq < fl[lanes[Lw].q_oldest].seq))
                Lw = L;
        if (Lw < 0) {
            if (done < npts) return fail(c, CHI0_EHIP, "solver stalled with unfinished points");
            break;
        }
        LaneState &ln = lanes[Lw];
        HIPCHK(c, hipEventSynchronize(c->step_ev[ln.q_oldest]));
        process(Lw, ln.q_oldest);
        ln.last_q = ln.q_oldest;
        ln.q_oldest ^= 1;
        --ln.n_inflight;
    }
    for (int L = 0; L < nl; ++L) CHK(issue_pending(L, lanes[L].last_q));   // alpha of the last points
    for (int L = 0; L < nl; ++L) HIPCHK(c, hipStreamSynchronize(c->lane_stream[L]));
    hipStream_t s = c->stream;
    if (Rst) launch_alpha_cross(t, s, n_omega, n_drive, P, Rst, Wst, alpha_dev);
    std::vector<double> ah((size_t)npts * n_drive * 2);
    HIPCHK(c, hipMemcpyAsync(ah.data(), alpha_dev, ah.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    int not_conv = 0;
    for (int w = 0; w < n_omega; ++w)
        for (int i = 0; i < n_drive; ++i) {
            const int p = w * n_drive + i;
            for (int k = 0; k < n_drive; ++k) {
                alpha[(((size_t)w * n_drive + k) * n_drive + i) * 2] = ah[((size_t)p * n_drive + k) * 2];
                alpha[(((size_t)w * n_drive + k) * n_drive + i) * 2 + 1] = ah[((size_t)p * n_drive + k) * 2 + 1];
            }
            if (!ps[p].converged) ++not_conv;
            if (stats) {
                chi0_point_stats &r = stats[p];
                r.iterations = ps[p].iters;
                r.restarts = ps[p].restarts;
                r.converged = ps[p].converged;
                r.breakdown = ps[p].breakdown;
                r.fallback = ps[p].fallback;
                r.warm_start = ps[p].warm;
                r.rel_residual = ps[p].rel;
                r.warm_rel0 = ps[p].warm_rel0;
                r.eps_x = ps[p].eps_x;
                r.eps_p = ps[p].eps_p;
                r.low_prec_steps = ps[p].low;
            }
        }
    c->err.clear();
    if (not_conv) {
        c->err = std::to_string(not_conv) + " point(s) did not reach the tolerance";
        return CHI0_NOT_CONVERGED;
    }
    return CHI0_OK;
}

extern "C" int chi0_solve_response(chi0_ctx *c, int32_t n_omega, const double *omega, double eps,
                                   int32_t n_drive, const double *V_ext, const chi0_solve_opts *opts,
                                   double *alpha, chi0_point_stats *stats) {
    return solve_impl(c, n_omega, omega, eps, n_drive, V_ext, opts, alpha, stats, nullptr);
}

extern "C" int chi0_solve_response_x(chi0_ctx *c, int32_t n_omega, const double *omega, double eps,
                                     int32_t n_drive, const double *V_ext, const chi0_solve_opts *opts,
                                     double *alpha, chi0_point_stats *stats, double *x) {
    if (!c) return CHI0_EINVAL;
    if (!x) return fail(c, CHI0_EINVAL, "NULL x");
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    if (n_omega <= 0 || n_drive < 1 || n_drive > 3)
        return solve_impl(c, n_omega, omega, eps, n_drive, V_ext, opts, alpha, stats, nullptr);
    HIPCHK(c, hipSetDevice(c->device));
    const int64_t npts = (int64_t)n_omega * n_drive;
    DevBuf xb;
    struct Guard { DevBuf *b; ~Guard() { b->release(); } } guard{&xb};
    double *xd = nullptr;
    CHK(dalloc(c, xb, &xd, npts * c->P_pad * 2));
    const int rc = solve_impl(c, n_omega, omega, eps, n_drive, V_ext, opts, alpha, stats, xd);
    if (rc < 0) return rc;
    HIPCHK(c, hipMemcpy2D(x, (size_t)c->P * 16, xd, (size_t)c->P_pad * 16, (size_t)c->P * 16, (size_t)npts,
                          hipMemcpyDeviceToHost));
    return rc;
}

// ----------------------------------------------------- warm-start fitting
namespace {
// Eigen-decomposition of a Hermitian n x n matrix (row-major, interleaved
// complex) by cyclic Jacobi rotations: A = V diag(w) V^H, w descending.
void jacobi_eigh(int n, std::vector<double> a, std::vector<double> &w, std::vector<double> &v) {
    auto re = [&](std::vector<double> &m, int i, int j) -> double & { return m[2 * ((size_t)i * n + j)]; };
    auto im = [&](std::vector<double> &m, int i, int j) -> double & { return m[2 * ((size_t)i * n + j) + 1]; };
    v.assign((size_t)2 * n * n, 0.0);
    for (int i = 0; i < n; ++i) re(v, i, i) = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = re(a, i, j) * re(a, i, j) + im(a, i, j) * im(a, i, j);
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double br = re(a, p, q), bi = im(a, p, q);
                const double bb = std::sqrt(br * br + bi * bi);
                if (bb <= 1e-300) continue;
                const double er = br / bb, ei = bi / bb;      // e^{i phi}
                const double app = re(a, p, p), aqq = re(a, q, q);
                const double tau = (aqq - app) / (2.0 * bb);
                const double tt = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double cc = 1.0 / std::sqrt(1.0 + tt * tt), ss = tt * cc;
                // U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] acting on columns p, q
                for (int k = 0; k < n; ++k) {     // A <- A U
                    const double xr = re(a, k, p), xi = im(a, k, p), yr = re(a, k, q), yi = im(a, k, q);
                    const double ur = yr * er + yi * ei, ui = yi * er - yr * ei;   // y e^{-i phi}
                    re(a, k, p) = cc * xr - ss * ur;
                    im(a, k, p) = cc * xi - ss * ui;
                    re(a, k, q) = ss * xr + cc * ur;
                    im(a, k, q) = ss * xi + cc * ui;
                }
                for (int k = 0; k < n; ++k) {     // A <- U^H A
                    const double xr = re(a, p, k), xi = im(a, p, k), yr = re(a, q, k), yi = im(a, q, k);
                    const double ur = yr * er - yi * ei, ui = yi * er + yr * ei;   // y e^{+i phi}
                    re(a, p, k) = cc * xr - ss * ur;
                    im(a, p, k) = cc * xi - ss * ui;
                    re(a, q, k) = ss * xr + cc * ur;
                    im(a, q, k) = ss * xi + cc * ui;
                }
                for (int k = 0; k < n; ++k) {     // V <- V U
                    const double xr = re(v, k, p), xi = im(v, k, p), yr = re(v, k, q), yi = im(v, k, q);
                    const double ur = yr * er + yi * ei, ui = yi * er - yr * ei;
                    re(v, k, p) = cc * xr - ss * ur;
                    im(v, k, p) = cc * xi - ss * ui;
                    re(v, k, q) = ss * xr + cc * ur;
                    im(v, k, q) = ss * xi + cc * ui;
                }
                im(a, p, p) = 0.0;
                im(a, q, q) = 0.0;
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return re(a, x, x) > re(a, y, y); });
    std::vector<double> vs((size_t)2 * n * n);
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        w[k] = re(a, idx[k], idx[k]);
        for (int i = 0; i < n; ++i) {
            vs[2 * ((size_t)i * n + k)] = re(v, i, idx[k]);
            vs[2 * ((size_t)i * n + k) + 1] = im(v, i, idx[k]);
        }
    }
    v.swap(vs);
}

uint64_t splitmix(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

extern "C" void chi0_ws_cfg_default(chi0_ws_cfg *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->rank = 64;
    cfg->width = 256;
    cfg->n_freq = 16;
    cfg->epochs = 3000;
    cfg->lr = 2e-3;
    cfg->seed = 1234;
    cfg->batch = 64;
    cfg->tol = 1e-10;
}

extern "C" void chi0_ws_free(chi0_ws *ws) {
    if (!ws) return;
    if (ws->ctx && ws->ctx->device >= 0) {
        (void)hipSetDevice(ws->ctx->device);
        (void)hipDeviceSynchronize();
    }
    delete ws;
}

static int ws_alloc(chi0_ctx *c, chi0_ws *w, int r, int width, int nf) {
    w->r = r;
    w->W = width;
    w->nf = nf;
    w->F = 2 * nf;
    w->O = (int)round_up(2 * r, 32);
    w->oW1 = 0;
    w->ob1 = w->oW1 + (int64_t)w->W * w->F;
    w->oW2 = w->ob1 + w->W;
    w->ob2 = w->oW2 + (int64_t)w->W * w->W;
    w->oW3 = w->ob2 + w->W;
    w->ob3 = w->oW3 + (int64_t)w->O * w->W;
    w->n_params = w->ob3 + w->O;
    DevBuf &b = w->buf;
    const int R = kMaxBatch;
    CHK(dalloc(c, b, &w->U, (int64_t)r * c->P_pad * 2));
    CHK(dalloc(c, b, &w->params, w->n_params));
    CHK(dalloc(c, b, &w->grads, w->n_params));
    CHK(dalloc(c, b, &w->am, w->n_params));
    CHK(dalloc(c, b, &w->av, w->n_params));
    CHK(dalloc(c, b, &w->mean, w->O));
    CHK(dalloc(c, b, &w->sdev, w->O));
    CHK(dalloc(c, b, &w->phi, (int64_t)R * w->F));
    CHK(dalloc(c, b, &w->H1, (int64_t)R * w->W));
    CHK(dalloc(c, b, &w->H2, (int64_t)R * w->W));
    CHK(dalloc(c, b, &w->dH1, (int64_t)R * w->W));
    CHK(dalloc(c, b, &w->dH2, (int64_t)R * w->W));
    CHK(dalloc(c, b, &w->out, (int64_t)R * w->O));
    CHK(dalloc(c, b, &w->dout, (int64_t)R * w->O));
    CHK(dalloc(c, b, &w->tgt, (int64_t)R * w->O));
    CHK(dalloc(c, b, &w->loss, 1 + 100000));
    CHK(dalloc(c, b, &w->omega_dev, R));
    CHK(dalloc(c, b, &w->jobs_dev, R));
    HIPCHK(c, hipDeviceSynchronize());
    return CHI0_OK;
}

static void ws_init_params(chi0_ws *w, uint64_t seed, std::vector<float> &h) {
    h.assign((size_t)w->n_params, 0.f);
    uint64_t st = seed;
    auto fill = [&](int64_t off, int rows, int cols) {   // Glorot uniform
        const double a = std::sqrt(6.0 / (rows + cols));
        for (int64_t i = 0; i < (int64_t)rows * cols; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            h[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(w->oW1, w->W, w->F);
    fill(w->oW2, w->W, w->W);
    fill(w->oW3, w->O, w->W);
}

extern "C" int chi0_ws_fit(chi0_ctx *c, int32_t n_train, const double *omega_train, double eps,
                           const double *drive, const chi0_ws_cfg *cfg_in, chi0_ws **out) {
    if (!out) return fail(c, CHI0_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    chi0_ws_cfg cfg;
    chi0_ws_cfg_default(&cfg);
    if (cfg_in) cfg = *cfg_in;
    if (n_train < 2 || n_train > kMaxBatch) return fail(c, CHI0_EINVAL, "n_train must be in [2, 256]");
    if (!omega_train || !drive) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (cfg.rank < 1 || cfg.rank > n_train) return fail(c, CHI0_EINVAL, "rank must be in [1, n_train]");
    if (cfg.width < 32 || cfg.width % 32 || cfg.width > 1024) return fail(c, CHI0_EINVAL, "width must be a multiple of 32 in [32, 1024]");
    if (cfg.n_freq != 16 && cfg.n_freq != 32) return fail(c, CHI0_EINVAL, "n_freq must be 16 or 32");
    if (cfg.epochs < 1 || cfg.epochs > 100000) return fail(c, CHI0_EINVAL, "epochs must be in [1, 100000]");
    if (!(cfg.lr > 0.0)) return fail(c, CHI0_EINVAL, "lr must be > 0");
    for (int i = 0; i < 4; ++i)
        if (cfg.reserved[i] != 0) return fail(c, CHI0_EINVAL, "reserved fields must be zero");
    if (!all_finite(omega_train, n_train)) return fail(c, CHI0_ENONFINITE, "non-finite omega_train");
    HIPCHK(c, hipSetDevice(c->device));
    const int P = c->P;
    const int64_t vlen = (int64_t)c->P_pad * 2;

    // 1. training solutions by plain FP64 GMRES (zero start)
    DevBuf tmp;
    struct Guard { DevBuf *b; ~Guard() { b->release(); } } guard{&tmp};
    double *S = nullptr, *G = nullptr, *Wc = nullptr;
    CHK(dalloc(c, tmp, &S, (int64_t)n_train * vlen));
    CHK(dalloc(c, tmp, &G, (int64_t)n_train * n_train * 2));
    chi0_solve_opts so;
    chi0_solve_opts_default(&so);
    so.restart = cfg.restart > 0 ? cfg.restart : std::min(P, 4000);
    so.tol = cfg.tol;
    so.batch = std::max(1, std::min(cfg.batch, n_train));
    so.max_iter = 20000;
    std::vector<double> al((size_t)n_train * 2);
    const int rc = solve_impl(c, n_train, omega_train, eps, 1, drive, &so, al.data(), nullptr, S);
    if (rc < 0) return rc;

    // 2. Gram matrix on the GPU, eigen-decomposition on the host (n_train <= 256)
    launch_gram(c->stream, n_train, S, vlen, P, G);
    std::vector<double> gh((size_t)n_train * n_train * 2);
    HIPCHK(c, hipMemcpyAsync(gh.data(), G, gh.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> lam, V;
    jacobi_eigh(n_train, gh, lam, V);
    int r = 0;
    while (r < cfg.rank && lam[r] > 1e-20 * lam[0] && lam[r] > 0.0) ++r;
    if (r < 1) return fail(c, CHI0_EINVAL, "training solutions are zero");

    chi0_ws *w = new (std::nothrow) chi0_ws();
    if (!w) return fail(c, CHI0_ENOMEM, "host allocation failed");
    std::unique_ptr<chi0_ws> hold(w);
    w->ctx = c;
    CHK(ws_alloc(c, w, r, cfg.width, cfg.n_freq));
    double wmax = 0.0;
    for (int i = 0; i < n_train; ++i) wmax = std::max(wmax, std::fabs(omega_train[i]));
    w->w_scale = cfg.w_scale > 0.0 ? cfg.w_scale : (wmax > 0.0 ? wmax : 1.0);
    w->epochs = cfg.epochs;

    // 3. basis U = S V_r Sigma_r^-1 (GPU) and coordinates C = U^H S = Sigma^-1 V_r^H G (host)
    std::vector<double> wc((size_t)n_train * r * 2);
    for (int t2 = 0; t2 < n_train; ++t2)
        for (int k = 0; k < r; ++k) {
            const double sg = std::sqrt(lam[k]);
            wc[2 * ((size_t)t2 * r + k)] = V[2 * ((size_t)t2 * n_train + k)] / sg;
            wc[2 * ((size_t)t2 * r + k) + 1] = V[2 * ((size_t)t2 * n_train + k) + 1] / sg;
        }
    CHK(dalloc(c, tmp, &Wc, (int64_t)wc.size()));
    HIPCHK(c, hipMemcpy(Wc, wc.data(), wc.size() * 8, hipMemcpyHostToDevice));
    launch_basis(c->stream, n_train, r, S, vlen, P, Wc, w->U);
    // C[t][k] = sum_s conj(Wc[s][k]) G[s][t]
    const int O = w->O, rows = (int)round_up(n_train, 32);
    std::vector<double> C((size_t)n_train * 2 * r);
    for (int t2 = 0; t2 < n_train; ++t2)
        for (int k = 0; k < r; ++k) {
            double cr = 0.0, ci = 0.0;
            for (int s2 = 0; s2 < n_train; ++s2) {
                const double ar = wc[2 * ((size_t)s2 * r + k)], ai = -wc[2 * ((size_t)s2 * r + k) + 1];
                const double gr = gh[2 * ((size_t)s2 * n_train + t2)], gi = gh[2 * ((size_t)s2 * n_train + t2) + 1];
                cr += ar * gr - ai * gi;
                ci += ar * gi + ai * gr;
            }
            C[(size_t)t2 * 2 * r + 2 * k] = cr;
            C[(size_t)t2 * 2 * r + 2 * k + 1] = ci;
        }
    // normalised targets: (c - mean) / std per output
    std::vector<float> mean(O, 0.f), sdev(O, 1.f), tg((size_t)kMaxBatch * O, 0.f);
    for (int o2 = 0; o2 < 2 * r; ++o2) {
        double mu = 0.0, sq = 0.0;
        for (int t2 = 0; t2 < n_train; ++t2) mu += C[(size_t)t2 * 2 * r + o2];
        mu /= n_train;
        for (int t2 = 0; t2 < n_train; ++t2) {
            const double d = C[(size_t)t2 * 2 * r + o2] - mu;
            sq += d * d;
        }
        const double sd = std::sqrt(sq / n_train);
        mean[o2] = (float)mu;
        sdev[o2] = (float)(sd > 0.0 ? sd : 1.0);
        for (int t2 = 0; t2 < n_train; ++t2)
            tg[(size_t)t2 * O + o2] = (float)((C[(size_t)t2 * 2 * r + o2] - mu) / sdev[o2]);
    }
    HIPCHK(c, hipMemcpy(w->mean, mean.data(), O * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(w->sdev, sdev.data(), O * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(w->tgt, tg.data(), tg.size() * 4, hipMemcpyHostToDevice));
    std::vector<float> p0;
    ws_init_params(w, cfg.seed, p0);
    HIPCHK(c, hipMemcpy(w->params, p0.data(), p0.size() * 4, hipMemcpyHostToDevice));

    // 4. full-batch Adam, cosine-decayed learning rate
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(w->omega_dev, omega_train, sizeof(double) * n_train, hipMemcpyHostToDevice, s));
    launch_features(s, n_train, rows, w->omega_dev, w->nf, w->w_scale, w->phi);
    const int E = cfg.epochs;
    DevBuf lbuf;
    struct Guard2 { DevBuf *b; ~Guard2() { b->release(); } } guard2{&lbuf};
    float *lh = nullptr;
    CHK(dalloc(c, lbuf, &lh, E));
    for (int ep = 1; ep <= E; ++ep) {
        const double lr = cfg.lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * (ep - 1) / E)));
        ws_forward(w, s, rows);
        ws_backward(w, s, rows, n_train, 2 * r, lh + (ep - 1));
        launch_adam(s, w->n_params, w->params, w->grads, w->am, w->av, (float)lr, 0.9f, 0.999f, 1e-8f, ep);
    }
    w->loss_hist.resize(E);
    HIPCHK(c, hipMemcpyAsync(w->loss_hist.data(), lh, (size_t)E * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    *out = hold.release();
    c->err.clear();
    return rc;
}

extern "C" int chi0_ws_predict(chi0_ws *w, int32_t n, const double *omega, double *x0) {
    if (!w || !w->ctx) return CHI0_EINVAL;
    chi0_ctx *c = w->ctx;
    if (n < 0 || n > kMaxBatch) return fail(c, CHI0_EINVAL, "n must be in [0, 256]");
    if (n == 0) return CHI0_OK;
    if (!omega || !x0) return fail(c, CHI0_EINVAL, "NULL pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    std::vector<Job> jl(n);
    for (int i = 0; i < n; ++i) jl[i] = {i, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(w->jobs_dev, jl.data(), sizeof(Job) * n, hipMemcpyHostToDevice, s));
    CHK(ws_infer(w, s, n, omega));
    launch_ws_apply(s, w->jobs_dev, n, w->out, w->O, w->mean, w->sdev, w->r, w->U, (int64_t)c->P_pad * 2,
                    x0, (int64_t)c->P * 2, c->P);
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return CHI0_OK;
}

extern "C" int chi0_ws_loss_history(const chi0_ws *w, float *loss, int32_t cap) {
    if (!w || cap < 0 || (cap > 0 && !loss)) return CHI0_EINVAL;
    const int n = std::min<int>(cap, (int)w->loss_hist.size());
    for (int i = 0; i < n; ++i) loss[i] = w->loss_hist[i];
    return (int)w->loss_hist.size();
}

// ============================================================= test hooks
#include "chi0_debug.h"

extern "C" int chi0_debug_dims(const chi0_ctx *c, int64_t *d) {
    if (!c || !d) return CHI0_EINVAL;
    if (!c->has_system) return CHI0_ENOSYS;
    const int64_t v[10] = {c->N, c->No, c->Nv, c->P, c->N_pad, c->No_pad, c->Nv_pad, c->P_pad,
                           c->n_blk, c->nnzB};
    for (int i = 0; i < 10; ++i) d[i] = v[i];
    return CHI0_OK;
}

extern "C" int chi0_debug_read(chi0_ctx *c, int32_t which, void *host, int64_t bytes) {
    if (!c || !host || bytes < 0) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no device system");
    const OpWork &o = c->op[0];
    const int64_t nc = o.nc_cap, mcol = (int64_t)c->No_pad * nc;
    const void *src = nullptr;
    int64_t cap = 0;
    switch (which) {
        case CHI0_DBG_ZIN: src = o.Zin; cap = (int64_t)c->P_pad * nc * 8; break;
        case CHI0_DBG_DV: src = o.dV; cap = c->nnzB * nc * 8; break;
        case CHI0_DBG_TT: src = o.Tt; cap = (int64_t)c->N_pad * mcol * 8; break;
        case CHI0_DBG_AT: src = o.at; cap = (int64_t)c->Nv_pad * mcol * 8; break;
        case CHI0_DBG_UT: src = o.Ut; cap = (int64_t)c->N_pad * mcol * 8; break;
        case CHI0_DBG_W: src = o.W; cap = c->nnzB * nc * 8; break;
        case CHI0_DBG_YOUT: src = o.Yout; cap = (int64_t)c->P_pad * nc * 8; break;
        case CHI0_DBG_BLK_NA: src = c->bm.blk_na; cap = (int64_t)c->n_blk * 4; break;
        case CHI0_DBG_BLK_NB: src = c->bm.blk_nb; cap = (int64_t)c->n_blk * 4; break;
        case CHI0_DBG_BLK_ENT: src = c->bm.blk_ent; cap = (int64_t)c->n_blk * 8; break;
        default: return fail(c, CHI0_EINVAL, "unknown buffer");
    }
    if (!src || bytes > cap) return fail(c, CHI0_EINVAL, "buffer not allocated or too small");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(host, src, (size_t)bytes, hipMemcpyDeviceToHost));
    return CHI0_OK;
}

extern "C" int chi0_ws_debug_dims(const chi0_ws *w, int64_t *d, double *w_scale) {
    if (!w || !d) return CHI0_EINVAL;
    const int64_t v[7] = {w->r, w->F, w->W, w->O, w->n_params, w->nf, 0};
    for (int i = 0; i < 6; ++i) d[i] = v[i];
    if (w_scale) *w_scale = w->w_scale;
    return CHI0_OK;
}

extern "C" int chi0_ws_debug_params(chi0_ws *w, float *host, int64_t n, int32_t set) {
    if (!w || !host || n != w->n_params) return CHI0_EINVAL;
    chi0_ctx *c = w->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    if (set)
        HIPCHK(c, hipMemcpy(w->params, host, (size_t)n * 4, hipMemcpyHostToDevice));
    else
        HIPCHK(c, hipMemcpy(host, w->params, (size_t)n * 4, hipMemcpyDeviceToHost));
    return CHI0_OK;
}

extern "C" int chi0_ws_debug_loss_grad(chi0_ws *w, int32_t n, const double *omega, const float *target,
                                       float *loss, float *grads) {
    if (!w || !omega || !target || !loss || !grads || n < 1 || n > kMaxBatch) return CHI0_EINVAL;
    chi0_ctx *c = w->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int rows = (int)round_up(n, 32);
    std::vector<float> tg((size_t)rows * w->O, 0.f);
    std::copy(target, target + (size_t)n * w->O, tg.begin());
    HIPCHK(c, hipMemcpyAsync(w->tgt, tg.data(), tg.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(w->omega_dev, omega, sizeof(double) * n, hipMemcpyHostToDevice, s));
    launch_features(s, n, rows, w->omega_dev, w->nf, w->w_scale, w->phi);
    ws_forward(w, s, rows);
    ws_backward(w, s, rows, n, 2 * w->r, w->loss);
    HIPCHK(c, hipMemcpyAsync(loss, w->loss, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(grads, w->grads, (size_t)w->n_params * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return CHI0_OK;
}

extern "C" int chi0_debug_lz_passes(const chi0_ctx *c, int32_t *passes, double *b_pre, int32_t cap) {
    if (!c) return CHI0_EINVAL;
    const int n = (int)c->lz_pass_rec.size();
    const int nc = n > 0 ? (int)(c->lz_bpre_rec.size() / n) : 0;
    for (int j = 0; j < std::min(n, cap); ++j) {
        if (passes) passes[j] = c->lz_pass_rec[j];
        if (b_pre)
            for (int s = 0; s < nc; ++s) b_pre[(int64_t)j * nc + s] = c->lz_bpre_rec[(int64_t)j * nc + s];
    }
    return n;
}

extern "C" int chi0_debug_eigh(int32_t n, const double *A, double *w, double *V) {
    if (n < 1 || !A || !w || !V) return CHI0_EINVAL;
    std::vector<double> a(A, A + (size_t)2 * n * n), lam, vec;
    jacobi_eigh(n, a, lam, vec);
    std::copy(lam.begin(), lam.end(), w);
    std::copy(vec.begin(), vec.end(), V);
    return CHI0_OK;
}

// ====================================================== Lanczos in transition space
// The pole form of the response (Casida's equations): Om2 = D^2 + S V_t^T K V_t S
// on the (occupied, virtual) transitions, alpha(w) = c^T (Om2 - (w + i eps)^2)^-1 c
// with c = S V_t^T d.  The recursion's operator is the chi0 operator's own
// kernels composed the other way round: the back half (b3), (b4), (d) maps a
// transition vector to products, K multiplies, the front half (a), (b1), (b2)
// maps back to transitions.
namespace {

// Zin [P_pad][nc] -> at = V_t^T Zin (transition layout)
void lz_front(chi0_ctx *c, OpWork &o, hipStream_t s, int nc) {
    Tracer *t = &c->tracer;
    const WorkSizes &w = c->ws;
    const int64_t mcol = (int64_t)c->No_pad * nc;
    launch_vertex_gather(t, s, c->bm, c->n_blk, o.Zin, o.dV, nc, w);
    launch_occ_transform(t, s, c->bm, c->n_atoms, c->Xo, c->No_pad, o.dV, o.Tt, nc, w);
    launch_dgemm(t, s, "casida_front", c->Nv_pad, c->No16 * nc, c->N16, c->N_pad, c->Xvt, c->N_pad, o.Tt, (int)mcol, o.at,
                 (int)mcol, 2.0 * w.N * w.Nv * w.No * nc, 8.0 * (w.N * w.No * nc + w.Nv * w.No * nc + w.N * w.Nv),
                 o.gemm_scratch, o.gemm_scratch_n, &c->tuner);
}

// at (transition layout) -> Yout = V_t at [P_pad][nc]
void lz_back(chi0_ctx *c, OpWork &o, hipStream_t s, int nc) {
    Tracer *t = &c->tracer;
    const WorkSizes &w = c->ws;
    const int64_t mcol = (int64_t)c->No_pad * nc;
    launch_dgemm(t, s, "virt_back", c->N_pad, c->No16 * nc, c->Nv16, c->Nv_pad, c->Xv, c->Nv_pad, o.at, (int)mcol,
                 o.Ut, (int)mcol, 2.0 * w.N * w.Nv * w.No * nc,
                 8.0 * (w.Nv * w.No * nc + w.N * w.No * nc + w.N * w.Nv), o.gemm_scratch, o.gemm_scratch_n,
                 &c->tuner);
    launch_occ_back(t, s, c->bm, c->n_atoms, c->max_rows, c->Xo, c->No_pad, c->No16, o.Ut, o.W, nc, w);
    launch_vertex_contract(t, s, c->bm, c->n_blk, c->P, o.W, o.part, o.Yout, nc, w, c->max_nprod);
}

// the back half, then Zin = K Yout
void lz_back_k(chi0_ctx *c, OpWork &o, hipStream_t s, int nc) {
    lz_back(c, o, s, nc);
    launch_kmatvec_skinny(&c->tracer, s, c->P_pad, c->K, o.Yout, o.Zin, nc, (double)c->P);
}

// Eigenvalues of the symmetric tridiagonal matrix (d, e) and the first row of
// its eigenvector matrix, by implicit QR steps with the Wilkinson shift
// (Golub & Van Loan, the symmetric QR algorithm), each rotation applied to
// the first row only.  d: k diagonal entries, e: k - 1 off-diagonal entries
// (both overwritten); z: first components on return.  false if an unreduced
// block fails to split within 60 steps per eigenvalue.
bool tridiag_eig_first_row(int k, std::vector<double> &d, std::vector<double> &e, std::vector<double> &z) {
    const double u = 2.220446049250313e-16;
    z.assign(k, 0.0);
    z[0] = 1.0;
    e.resize(std::max(k - 1, 0));
    int hi = k - 1;
    int64_t iters = 0;
    const int64_t max_iters = 60 * (int64_t)std::max(k, 1);
    auto negligible = [&](int i) { return std::fabs(e[i]) <= u * (std::fabs(d[i]) + std::fabs(d[i + 1])); };
    while (hi > 0) {
        if (negligible(hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(lo - 1)) --lo;
        if (++iters > max_iters) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closer to d[hi]
        const double dd = 0.5 * (d[hi - 1] - d[hi]), eh = e[hi - 1];
        const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, eh);
        const double mu = d[hi] - eh * eh / den;
        // chase the bulge from (lo, lo+1) down to (hi-1, hi)
        double bulge = 0.0;
        for (int i = lo; i < hi; ++i) {
            double cth, sth;
            if (i == lo) {
                const double x = d[lo] - mu, y = e[lo], rho = std::hypot(x, y);
                cth = rho > 0.0 ? x / rho : 1.0;
                sth = rho > 0.0 ? -y / rho : 0.0;
            } else {
                const double x = e[i - 1], y = bulge, rho = std::hypot(x, y);
                cth = rho > 0.0 ? x / rho : 1.0;
                sth = rho > 0.0 ? -y / rho : 0.0;
                e[i - 1] = rho;
            }
            // [p r; r q] <- J^T [p r; r q] J with J = [c s; -s c]
            const double p = d[i], q = d[i + 1], r = e[i];
            const double cc = cth * cth, ss = sth * sth, cs = cth * sth;
            d[i] = cc * p - 2.0 * cs * r + ss * q;
            d[i + 1] = ss * p + 2.0 * cs * r + cc * q;
            e[i] = cs * (p - q) + (cc - ss) * r;
            if (i + 1 < hi) {
                bulge = -sth * e[i + 1];
                e[i + 1] = cth * e[i + 1];
            }
            const double z0 = z[i], z1 = z[i + 1];
            z[i] = cth * z0 - sth * z1;
            z[i + 1] = sth * z0 + cth * z1;
        }
    }
    return true;
}

struct DevScope {   // frees a call's device workspace on every exit
    DevBuf buf;
    ~DevScope() { buf.release(); }
};

}  // namespace

extern "C" void chi0_lanczos_opts_default(chi0_lanczos_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->k_max = 4000;
    o->reorth = CHI0_LZ_REORTH_PARTIAL;
    o->tol = 0.0;
    o->check_every = 100;
}

extern "C" int chi0_lanczos(chi0_ctx *c, int32_t n_drive, const double *drives, const chi0_lanczos_opts *opts,
                            double *a_out, double *b_out, double *cn2_out, int32_t *len_out) {
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    chi0_lanczos_opts o;
    if (opts)
        o = *opts;
    else
        chi0_lanczos_opts_default(&o);
    if (n_drive < 1 || n_drive > 4) return fail(c, CHI0_EINVAL, "n_drive must be 1..4");
    if (!drives || !a_out || !b_out || !cn2_out || !len_out) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (o.k_max < 1) return fail(c, CHI0_EINVAL, "k_max < 1");
    if (o.reorth < CHI0_LZ_REORTH_NONE || o.reorth > CHI0_LZ_REORTH_PARTIAL)
        return fail(c, CHI0_EINVAL, "unknown reorth");
    if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return fail(c, CHI0_EINVAL, "tol must be finite and >= 0");
    if (o.n_check < 0 || (o.n_check > 0 && !o.omega_check)) return fail(c, CHI0_EINVAL, "bad check frequencies");
    if (o.tol > 0.0 && (o.n_check == 0 || o.check_every < 1))
        return fail(c, CHI0_EINVAL, "tol > 0 needs check frequencies and check_every >= 1");
    if (o.n_check > 0 && (!(o.eps > 0.0) || !std::isfinite(o.eps)))
        return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (o.n_check > 0 && !all_finite(o.omega_check, o.n_check))
        return fail(c, CHI0_ENONFINITE, "non-finite check frequency");
    if (o.graph != 0 && o.graph != 1) return fail(c, CHI0_EINVAL, "graph must be 0 or 1");
    if (o.n_x < 0 || (o.n_x > 0 && (!o.omega_x || (!o.x && !o.alpha_x))))
        return fail(c, CHI0_EINVAL, "bad solution frequencies or outputs");
    if (o.n_x > 0 && o.reorth == CHI0_LZ_REORTH_NONE)
        return fail(c, CHI0_EINVAL, "solutions need the stored basis of a reorthogonalised recursion");
    if (o.n_x > 0 && (!(o.eps > 0.0) || !std::isfinite(o.eps)))
        return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (o.n_x > 0 && !all_finite(o.omega_x, o.n_x)) return fail(c, CHI0_ENONFINITE, "non-finite solution frequency");
    for (int32_t r : o.reserved)
        if (r != 0) return fail(c, CHI0_EINVAL, "reserved fields must be zero");
    const int P = c->P, nc = n_drive;
    if (!all_finite(drives, (int64_t)n_drive * P)) return fail(c, CHI0_ENONFINITE, "non-finite drive");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int kmax = (int)std::min<int64_t>(o.k_max, (int64_t)c->No * c->Nv);
    const bool ring = o.reorth == CHI0_LZ_REORTH_NONE;
    OpWork &ow = c->op[0];
    // the operator passes of the solutions carry 2 LZ_XCOL real columns
    CHK(ensure_ws(c, ow, std::max({nc, ow.nc_cap, o.n_x > 0 ? 2 * LZ_XCOL : 0})));

    const int64_t tp = (int64_t)c->No_pad * c->Nv_pad, tc = round_up((int64_t)c->No * c->Nv, 64), n = tc * nc;
    const int64_t nvec = ring ? 3 : (int64_t)kmax + 1;
    {
        size_t fr = 0, tot = 0;
        HIPCHK(c, hipMemGetInfo(&fr, &tot));
        const double need =
            8.0 * (double)(nvec * n + 2 * tc + 69 * ((int64_t)kmax + 2) * nc + (ring ? 0 : LZ_GROUPS * n) +
                           (o.n_x > 0 ? (int64_t)kmax * LZ_XCOL * 6 + (int64_t)P * (nc + 2 * LZ_XCOL) : 0));
        if (need > 0.9 * (double)fr)
            return fail(c, CHI0_ENOMEM, "the Lanczos basis does not fit in free device memory (k_max too large "
                                        "for full reorthogonalisation)");
    }
    DevScope ws;
    LanczosDev L{};
    double *St = nullptr, *D2t = nullptr, *part2 = nullptr, *h = nullptr, *part3 = nullptr, *om = nullptr,
           *spec = nullptr;
    CHK(dalloc(c, ws.buf, &L.R, nvec * n));
    CHK(dalloc(c, ws.buf, &St, tc));
    CHK(dalloc(c, ws.buf, &D2t, tc));
    CHK(dalloc(c, ws.buf, &L.a, (int64_t)kmax * nc));
    CHK(dalloc(c, ws.buf, &L.b, (int64_t)kmax * nc));
    CHK(dalloc(c, ws.buf, &L.cn2, nc));
    CHK(dalloc(c, ws.buf, &L.len, nc));
    CHK(dalloc(c, ws.buf, &L.step, 1));
    CHK(dalloc(c, ws.buf, &L.part, (int64_t)LZ_BLOCKS * nc));
    if (!ring) {
        CHK(dalloc(c, ws.buf, &part2, (int64_t)64 * (kmax + 1) * nc));
        CHK(dalloc(c, ws.buf, &h, (int64_t)(kmax + 1) * nc));
        CHK(dalloc(c, ws.buf, &part3, (int64_t)LZ_GROUPS * n));
    }
    double *xdw = nullptr, *xY = nullptr, *xom = nullptr, *xdrv = nullptr, *xrows = nullptr, *xalpha = nullptr;
    if (o.n_x > 0) {
        CHK(dalloc(c, ws.buf, &xdw, (int64_t)kmax * LZ_XCOL * 4));
        CHK(dalloc(c, ws.buf, &xY, (int64_t)kmax * LZ_XCOL * 2));
        CHK(dalloc(c, ws.buf, &xom, LZ_XCOL));
        CHK(dalloc(c, ws.buf, &xdrv, (int64_t)nc * P));
        CHK(dalloc(c, ws.buf, &xrows, (int64_t)LZ_XCOL * P * 2));
        CHK(dalloc(c, ws.buf, &xalpha, (int64_t)LZ_XCOL * nc * 2));
        HIPCHK(c, hipMemcpy(xdrv, drives, (size_t)nc * P * 8, hipMemcpyHostToDevice));
    }
    if (o.n_check > 0) {
        CHK(dalloc(c, ws.buf, &om, o.n_check));
        CHK(dalloc(c, ws.buf, &spec, 2 * (int64_t)o.n_check * nc));
        HIPCHK(c, hipMemcpyAsync(om, o.omega_check, (size_t)o.n_check * 8, hipMemcpyHostToDevice, s));
    }
    L.n = n;
    L.tc = tc;
    L.tp = tp;
    L.t_alg = (int64_t)c->No * c->Nv;
    L.no = c->No;
    L.nv = c->Nv;
    L.no_pad = c->No_pad;
    L.ring = ring ? 1 : 0;
    L.passes = ring ? 0 : (o.reorth == CHI0_LZ_REORTH_FULL2 ? 2 : 1);   // PARTIAL: 1 where it reorthogonalises
    L.nc = nc;
    L.kmax = kmax;
    L.St = St;
    L.D2t = D2t;
    L.at = ow.at;
    launch_zero(&c->tracer, s, L.a, (int64_t)kmax * nc);
    launch_zero(&c->tracer, s, L.b, (int64_t)kmax * nc);
    launch_lz_tables(s, c->Dlt, c->No, c->Nv, c->Nv_pad, tc, c->occ, St, D2t);
    // drives -> Zin [P_pad][nc] (padding rows zero), c = S V_t^T d
    {
        std::vector<double> zin((size_t)c->P_pad * nc, 0.0);
        for (int sq = 0; sq < nc; ++sq)
            for (int mu = 0; mu < P; ++mu) zin[(size_t)mu * nc + sq] = drives[(size_t)sq * P + mu];
        launch_zero(&c->tracer, s, ow.Yout, (int64_t)c->P_pad * nc);
        HIPCHK(c, hipMemcpyAsync(ow.Zin, zin.data(), zin.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));   // zin is a host temporary
    }
    lz_front(c, ow, s, nc);
    launch_lz_start(&c->tracer, s, L);

    // convergence checks on the host: alpha_k at the check frequencies
    std::vector<double> cur(2 * (size_t)o.n_check * nc), prev;
    std::vector<int> lenh(nc);
    int met = 0;
    bool converged = false;
    auto check = [&](int k) -> int {
        launch_lz_cfrac(s, L.a, L.b, nc, k, L.len, L.cn2, om, o.n_check, o.eps, spec);
        HIPCHK(c, hipMemcpyAsync(cur.data(), spec, cur.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(lenh.data(), L.len, nc * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        double worst = 0.0;
        if (!prev.empty()) {
            for (int sq = 0; sq < nc; ++sq) {
                double mx = 0.0;
                for (int i = 0; i < o.n_check; ++i) mx = std::max(mx, std::fabs(cur[2 * ((size_t)i * nc + sq) + 1]));
                const double floor_v = std::max(1e-3 * mx, 1e-300);
                for (int i = 0; i < o.n_check; ++i) {
                    const size_t q = 2 * ((size_t)i * nc + sq);
                    const double dr = cur[q] - prev[q], di = cur[q + 1] - prev[q + 1];
                    const double den = std::max(std::fabs(cur[q + 1]), floor_v);
                    worst = std::max(worst, std::hypot(dr, di) / den);
                }
            }
            met = worst <= o.tol ? met + 1 : 0;
        }
        prev = cur;
        return CHI0_OK;
    };

    hipGraphExec_t exec = nullptr;
    struct ExecScope {
        hipGraphExec_t *e;
        ~ExecScope() {
            if (*e) (void)hipGraphExecDestroy(*e);
        }
    } exec_scope{&exec};
    const bool use_graph = o.graph == 1 && ring && !c->tracer.on;
    // partial reorthogonalisation: the estimates and the decision live on the device
    const bool partial = o.reorth == CHI0_LZ_REORTH_PARTIAL;
    int *flag_h = nullptr;
    struct PinScope {
        int **p;
        ~PinScope() {
            if (*p) (void)hipHostFree(*p);
        }
    } pin_scope{&flag_h};
    if (partial) {
        CHK(dalloc(c, ws.buf, &L.omega, 3 * (int64_t)nc * (kmax + 2)));
        CHK(dalloc(c, ws.buf, &L.anorm, nc));
        CHK(dalloc(c, ws.buf, &L.flag, 2));
        const double one = 1.0;
        for (int sq = 0; sq < nc; ++sq)   // row 0: q_0 . q_0 = 1
            HIPCHK(c, hipMemcpy(L.omega + (int64_t)sq * (kmax + 2), &one, 8, hipMemcpyHostToDevice));
        if (c->tracer.on) HIPCHK(c, hipHostMalloc((void **)&flag_h, sizeof(int), 0));
    }
    c->lz_pass_rec.clear();
    c->lz_bpre_rec.clear();
    int steps = 0;
    for (int j = 0; j < kmax; ++j) {
        if (partial) {
            lz_back_k(c, ow, s, nc);
            lz_front(c, ow, s, nc);
            if (c->tracer.on) {
                // per-kernel timing: read the decision, so that the pass is launched
                // (and counted) only where it runs; same arithmetic as the gated launch
                launch_lz_step_head(&c->tracer, s, L, j);
                HIPCHK(c, hipMemcpyAsync(flag_h, L.flag, sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(c, hipStreamSynchronize(s));
                c->lz_pass_rec.push_back(*flag_h ? 1 : 0);
                c->lz_bpre_rec.resize(c->lz_bpre_rec.size() + nc);
                HIPCHK(c, hipMemcpy(c->lz_bpre_rec.data() + c->lz_bpre_rec.size() - nc, L.b + (int64_t)j * nc,
                                    sizeof(double) * nc, hipMemcpyDeviceToHost));
                launch_lz_step_tail(&c->tracer, s, L, j, *flag_h ? 1 : 0, part2, h, part3);
            } else {
                launch_lz_step_partial(&c->tracer, s, L, j, part2, h, part3);
            }
        } else if (use_graph && j >= 1) {
            if (!exec) {   // capture one step (the GEMM tiles were tuned by step 0)
                if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                HIPCHK(c, hipStreamSynchronize(s));
                hipGraph_t g = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                lz_back_k(c, ow, c->cap_stream, nc);
                lz_front(c, ow, c->cap_stream, nc);
                launch_lz_step(&c->tracer, c->cap_stream, L, j, part2, h, part3);
                HIPCHK(c, hipStreamEndCapture(c->cap_stream, &g));
                const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    exec = nullptr;
                    return fail(c, CHI0_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                }
            }
            HIPCHK(c, hipGraphLaunch(exec, s));
        } else {
            lz_back_k(c, ow, s, nc);
            lz_front(c, ow, s, nc);
            launch_lz_step(&c->tracer, s, L, j, part2, h, part3);
        }
        steps = j + 1;
        const bool last = steps == kmax;
        if (o.n_check > 0 && (steps % std::max(o.check_every, 1) == 0 || last)) {
            CHK(check(steps));
            bool all_ended = true;
            for (int sq = 0; sq < nc; ++sq) all_ended = all_ended && lenh[sq] < kmax && lenh[sq] <= steps;
            if (all_ended || (o.tol > 0.0 && met >= 2)) {
                converged = true;
                break;
            }
        }
    }
    HIPCHK(c, hipGetLastError());
    std::vector<double> ah((size_t)kmax * nc), bh((size_t)kmax * nc), cn2h(nc);
    HIPCHK(c, hipMemcpyAsync(ah.data(), L.a, ah.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(bh.data(), L.b, bh.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(cn2h.data(), L.cn2, nc * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(lenh.data(), L.len, nc * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    bool all_ended = true;
    for (int sq = 0; sq < nc; ++sq) {
        const int ln = std::min(lenh[sq], steps);
        all_ended = all_ended && lenh[sq] <= steps && lenh[sq] < kmax;
        len_out[sq] = ln;
        cn2_out[sq] = cn2h[sq];
        for (int j = 0; j < o.k_max; ++j) {
            a_out[(size_t)sq * o.k_max + j] = j < ln ? ah[(size_t)j * nc + sq] : 0.0;
            b_out[(size_t)sq * o.k_max + j] = j < ln ? bh[(size_t)j * nc + sq] : 0.0;
        }
    }
    if (o.n_x > 0) {
        // solutions of eq. sle from the stored basis, W frequencies per operator pass
        int kuse = 0;
        for (int sq = 0; sq < nc; ++sq) kuse = std::max(kuse, std::min(lenh[sq], steps));
        const int W = LZ_XCOL / nc, M = W * nc;
        std::vector<double> omb(W);
        for (int p0 = 0; p0 < o.n_x; p0 += W) {
            const int nw = std::min(W, o.n_x - p0);
            for (int w = 0; w < W; ++w) omb[w] = o.omega_x[p0 + std::min(w, nw - 1)];
            HIPCHK(c, hipMemcpyAsync(xom, omb.data(), W * 8, hipMemcpyHostToDevice, s));
            if (kuse > 0) {
                launch_lz_solution_cols(&c->tracer, s, L, kuse, L.len, xom, nw, o.eps, xdw, xY, ow.at);
                lz_back(c, ow, s, 2 * M);
            } else {
                launch_zero(&c->tracer, s, ow.Yout, (int64_t)c->P_pad * 2 * M);
            }
            launch_lz_solution_out(s, ow.Yout, nc, nw, P, xdrv, o.x ? xrows : nullptr, o.alpha_x ? xalpha : nullptr);
            if (o.x)
                HIPCHK(c, hipMemcpyAsync(o.x + (size_t)p0 * nc * P * 2, xrows, (size_t)nw * nc * P * 16,
                                         hipMemcpyDeviceToHost, s));
            if (o.alpha_x)
                HIPCHK(c, hipMemcpyAsync(o.alpha_x + (size_t)p0 * nc * nc * 2, xalpha, (size_t)nw * nc * nc * 16,
                                         hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
        }
        HIPCHK(c, hipGetLastError());
    }
    if (o.tol > 0.0 && !converged && !all_ended) return CHI0_NOT_CONVERGED;
    return CHI0_OK;
}

extern "C" int chi0_lanczos_spectrum(chi0_ctx *c, int32_t n_drive, int32_t ld, const double *a, const double *b,
                                     const double *cn2, const int32_t *len, int32_t n_omega, const double *omega,
                                     double eps, double *alpha) {
    if (!c) return CHI0_EINVAL;
    if (c->device < 0) return fail(c, CHI0_ENOSYS, "host-only context");
    if (n_drive < 1 || ld < 0 || n_omega < 0) return fail(c, CHI0_EINVAL, "bad sizes");
    if (n_omega == 0) return CHI0_OK;
    if (!a || !b || !cn2 || !len || !omega || !alpha) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    int kuse = 0;
    for (int sq = 0; sq < n_drive; ++sq) {
        if (len[sq] < 0 || len[sq] > ld) return fail(c, CHI0_EINVAL, "len outside 0..ld");
        kuse = std::max(kuse, (int)len[sq]);
    }
    if (!all_finite(omega, n_omega) || !all_finite(cn2, n_drive)) return fail(c, CHI0_ENONFINITE, "non-finite input");
    std::vector<double> ad((size_t)std::max(kuse, 1) * n_drive, 0.0), bd(ad.size(), 0.0);
    for (int sq = 0; sq < n_drive; ++sq)
        for (int j = 0; j < len[sq]; ++j) {
            ad[(size_t)j * n_drive + sq] = a[(size_t)sq * ld + j];
            bd[(size_t)j * n_drive + sq] = b[(size_t)sq * ld + j];
        }
    if (!all_finite(ad.data(), (int64_t)ad.size()) || !all_finite(bd.data(), (int64_t)bd.size()))
        return fail(c, CHI0_ENONFINITE, "non-finite coefficient");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    DevScope ws;
    double *a_d = nullptr, *b_d = nullptr, *c_d = nullptr, *om_d = nullptr, *out_d = nullptr;
    int *len_d = nullptr;
    CHK(dalloc(c, ws.buf, &a_d, (int64_t)ad.size()));
    CHK(dalloc(c, ws.buf, &b_d, (int64_t)bd.size()));
    CHK(dalloc(c, ws.buf, &c_d, n_drive));
    CHK(dalloc(c, ws.buf, &len_d, n_drive));
    CHK(dalloc(c, ws.buf, &om_d, n_omega));
    CHK(dalloc(c, ws.buf, &out_d, 2 * (int64_t)n_omega * n_drive));
    HIPCHK(c, hipMemcpyAsync(a_d, ad.data(), ad.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(b_d, bd.data(), bd.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c_d, cn2, (size_t)n_drive * 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(len_d, len, (size_t)n_drive * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(om_d, omega, (size_t)n_omega * 8, hipMemcpyHostToDevice, s));
    launch_lz_cfrac(s, a_d, b_d, n_drive, kuse, len_d, c_d, om_d, n_omega, eps, out_d);
    HIPCHK(c, hipMemcpyAsync(alpha, out_d, 2 * (size_t)n_omega * n_drive * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return CHI0_OK;
}

extern "C" int chi0_lanczos_poles(int32_t k, const double *a, const double *b, double c_norm2, double *theta,
                                  double *resid) {
    if (k < 1 || !a || !b || !theta || !resid) return CHI0_EINVAL;
    if (!all_finite(a, k) || (k > 1 && !all_finite(b, k - 1)) || !std::isfinite(c_norm2)) return CHI0_ENONFINITE;
    if (c_norm2 < 0.0) return CHI0_EINVAL;
    std::vector<double> d(a, a + k), e(b, b + (k - 1)), z;
    if (!tridiag_eig_first_row(k, d, e, z)) return CHI0_NOT_CONVERGED;
    std::vector<int> order(k);
    for (int i = 0; i < k; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int i = 0; i < k; ++i) {
        theta[i] = d[order[i]];
        resid[i] = c_norm2 * z[order[i]] * z[order[i]];
    }
    return CHI0_OK;
}

// ============================================================ two-sided Lanczos
// chi0_solve_bilanczos: one recursion per (omega, drive) point, up to kBlBatch
// points at once.  Per step: K v, then chi0 over [K v, w] (two complex
// columns per point, each point at its own frequency), then K chi0 w, then
// the per-point vector work (kernels_bilanczos.hip).  The coefficients stay
// on the device; every kBlCheck steps the host copies the new ones and runs,
// per point, the LDL^T recurrences of T_k (no pivoting):
//   d_1 = alpha_1,  d_j = alpha_j - beta_j^2 / d_{j-1},
//   z_1 = 1,        z_j = -(beta_j / d_{j-1}) z_{j-1},
//   P_k = beta_1^2 sum_{j <= k} z_j^2 / d_j          (= beta_1^2 e_1^T T_k^-1 e_1),
//   e_k^T T_k^-1 beta_1 e_1 = beta_1 z_k / d_k,
// so the residual |b - A x_k| = |beta_1 z_k / d_k| |r_k| costs O(1) per step.
namespace {
constexpr int kBlBatch = 64;   // points per batch: 128 complex chi0 columns per step
constexpr int kBlCheck = 10;   // steps between host checks

struct BlPoint {
    double d_r = 0, d_i = 0, z_r = 1, z_i = 0, P_r = 0, P_i = 0;
    int steps = 0, status = 1;
    bool done = false;
};
}  // namespace

extern "C" int chi0_solve_bilanczos(chi0_ctx *c, int32_t n_omega, const double *omega, double eps, int32_t n_drive,
                                    const double *drives, double tol, int32_t max_steps, double *alpha,
                                    int32_t *steps, int32_t *status) {
    if (!c) return CHI0_EINVAL;
    if (!c->has_system || c->device < 0) return fail(c, CHI0_ENOSYS, "no system on a device context");
    if (n_omega < 0) return fail(c, CHI0_EINVAL, "n_omega < 0");
    if (n_drive < 1 || n_drive > 3) return fail(c, CHI0_EINVAL, "n_drive must be 1..3");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(c, CHI0_EINVAL, "eps must be finite and > 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(c, CHI0_EINVAL, "tol must be finite and > 0");
    if (max_steps < 1) return fail(c, CHI0_EINVAL, "max_steps < 1");
    if ((int64_t)n_omega * n_drive > INT32_MAX) return fail(c, CHI0_EINVAL, "too many points");
    if (n_omega == 0) return CHI0_OK;
    if (!omega || !drives || !alpha) return fail(c, CHI0_EINVAL, "NULL pointer");
    if (!all_finite(omega, n_omega)) return fail(c, CHI0_ENONFINITE, "non-finite omega");
    const int P = c->P, P_pad = c->P_pad;
    if (!all_finite(drives, (int64_t)n_drive * P)) return fail(c, CHI0_ENONFINITE, "non-finite drive");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    Tracer *t = &c->tracer;
    const int npt = n_omega * n_drive;
    const int NB = std::min(npt, kBlBatch);
    const int ms = max_steps;
    OpWork &ow = c->op[0];
    CHK(ensure_ws(c, ow, std::max(4 * NB, ow.nc_cap)));
    {
        size_t fr = 0, tot = 0;
        HIPCHK(c, hipMemGetInfo(&fr, &tot));
        const double need = 8.0 * ((double)P_pad * 2 * NB * 7 + (double)n_drive * P_pad + 5.0 * NB * (ms + 1));
        if (need > 0.9 * (double)fr) return fail(c, CHI0_ENOMEM, "the recursion's workspace does not fit (max_steps?)");
    }
    DevScope ws;
    double *D = nullptr, *V[2] = {}, *W[2] = {}, *KV = nullptr, *CW = nullptr, *KCW = nullptr, *om2 = nullptr;
    double *al = nullptr, *be = nullptr, *rn = nullptr, *bn = nullptr;
    int *flag = nullptr;
    const int64_t vn = (int64_t)P_pad * 2 * NB;
    CHK(dalloc(c, ws.buf, &D, (int64_t)n_drive * P_pad));
    for (int i = 0; i < 2; ++i) {
        CHK(dalloc(c, ws.buf, &V[i], vn));
        CHK(dalloc(c, ws.buf, &W[i], vn));
    }
    CHK(dalloc(c, ws.buf, &KV, vn));
    CHK(dalloc(c, ws.buf, &CW, vn));
    CHK(dalloc(c, ws.buf, &KCW, vn));
    CHK(dalloc(c, ws.buf, &om2, 2 * NB));
    const int ldal = 2 * ms, ldbe = 2 * (ms + 1), ldrn = ms;
    CHK(dalloc(c, ws.buf, &al, (int64_t)NB * ldal));
    CHK(dalloc(c, ws.buf, &be, (int64_t)NB * ldbe));
    CHK(dalloc(c, ws.buf, &rn, (int64_t)NB * ldrn));
    CHK(dalloc(c, ws.buf, &bn, NB));
    CHK(dalloc(c, ws.buf, &flag, NB));
    {
        std::vector<double> dh((size_t)n_drive * P_pad, 0.0);
        for (int i = 0; i < n_drive; ++i)
            std::copy(drives + (size_t)i * P, drives + (size_t)(i + 1) * P, dh.begin() + (size_t)i * P_pad);
        HIPCHK(c, hipMemcpy(D, dh.data(), dh.size() * 8, hipMemcpyHostToDevice));
    }
    auto kprod = [&](const double *X, double *Y, int nc) {
        if (nc <= 32)
            launch_kmatvec_skinny(t, s, P_pad, c->K, X, Y, nc, (double)P);
        else
            launch_dgemm(t, s, "kernel_matmul", P_pad, nc, P_pad, P_pad, c->K, P_pad, X, nc, Y, nc,
                         2.0 * P * (double)P * nc, 8.0 * ((double)P * P + 2.0 * P * nc), ow.gemm_scratch,
                         ow.gemm_scratch_n, &c->tuner);
    };
    std::vector<double> omh(2 * NB), alh((size_t)NB * ldal), beh((size_t)NB * ldbe), rnh((size_t)NB * ldrn),
        bnh(NB);
    std::vector<int> flh(NB);
    // pinned staging of the device-to-host copies: the new coefficients of a check
    // window (at most kBlCheck steps), the start values and the flags
    struct Pinned {
        void *p = nullptr;
        ~Pinned() {
            if (p) (void)hipHostFree(p);
        }
    } pin;
    const size_t n_al = (size_t)NB * 2 * kBlCheck, n_be = (size_t)NB * 2 * kBlCheck, n_rn = (size_t)NB * kBlCheck;
    HIPCHK(c, hipHostMalloc(&pin.p, (n_al + n_be + n_rn + 2 * (size_t)NB) * 8, 0));
    double *s_al = static_cast<double *>(pin.p), *s_be = s_al + n_al, *s_rn = s_be + n_be, *s_bn = s_rn + n_rn;
    int *s_fl = reinterpret_cast<int *>(s_bn + NB);
    int rc = CHI0_OK;
    for (int p0 = 0; p0 < npt; p0 += NB) {
        const int np = std::min(NB, npt - p0);
        const int nc = 2 * np;   // real columns of one vector per point
        for (int q = 0; q < np; ++q) omh[q] = omh[np + q] = omega[(p0 + q) / n_drive];
        HIPCHK(c, hipMemcpyAsync(om2, omh.data(), (size_t)2 * np * 8, hipMemcpyHostToDevice, s));
        // b = chi0 d, then the start vectors
        launch_bl_drives(s, P, P_pad, np, p0, n_drive, D, ow.Zin);
        run_chi0(c, ow, s, np, eps, CHI0_PREC_FP64, om2, t, &c->tuner);
        launch_bl_init(s, P, np, p0, n_drive, D, P_pad, ow.Yout, nc, V[0], W[0], V[1], W[1], nc, be, ldbe, bn, flag);
        HIPCHK(c, hipMemcpyAsync(s_fl, flag, (size_t)np * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(s_bn, bn, (size_t)np * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpy2DAsync(s_be, 16, be, ldbe * 8, 16, np, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        HIPCHK(c, hipGetLastError());
        for (int q = 0; q < np; ++q) {
            flh[q] = s_fl[q];
            bnh[q] = s_bn[q];
            beh[(size_t)q * ldbe] = s_be[2 * q];
            beh[(size_t)q * ldbe + 1] = s_be[2 * q + 1];
        }
        std::vector<BlPoint> pt(np);
        int active = 0;
        for (int q = 0; q < np; ++q) {
            if (flh[q] == -1) {   // zero right-hand side: x = 0; else d^T chi0 d = 0 before any step
                pt[q].done = true;
                pt[q].status = bnh[q] == 0.0 ? 0 : 2;
            } else {
                ++active;
            }
        }
        int cur = 0, k0 = 0;
        for (int k = 0; k < ms && active > 0; ++k) {
            kprod(V[cur], KV, nc);
            launch_bl_pack(s, P_pad, nc, KV, W[cur], ow.Zin);
            run_chi0(c, ow, s, 2 * np, eps, CHI0_PREC_FP64, om2, t, &c->tuner);
            launch_bl_unpack(s, P, P_pad, nc, ow.Yout, CW);
            kprod(CW, KCW, nc);
            launch_bl_step(s, np, P, k, ow.Yout, KCW, V[cur], W[cur], V[cur ^ 1], W[cur ^ 1], nc, al, ldal, be, ldbe,
                           rn, ldrn, flag);
            cur ^= 1;
            if ((k + 1) % kBlCheck != 0 && k + 1 != ms) continue;
            // the coefficients of steps k0..k
            const int nk = k - k0 + 1;
            HIPCHK(c, hipMemcpy2DAsync(s_al, (size_t)nk * 16, al + 2 * k0, ldal * 8, (size_t)nk * 16, np,
                                       hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpy2DAsync(s_be, (size_t)nk * 16, be + 2 * (k0 + 1), ldbe * 8, (size_t)nk * 16, np,
                                       hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpy2DAsync(s_rn, (size_t)nk * 8, rn + k0, ldrn * 8, (size_t)nk * 8, np,
                                       hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpyAsync(s_fl, flag, (size_t)np * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            HIPCHK(c, hipGetLastError());
            for (int q = 0; q < np; ++q) {
                std::copy(s_al + (size_t)q * 2 * nk, s_al + (size_t)(q + 1) * 2 * nk, alh.begin() + (size_t)q * ldal + 2 * k0);
                std::copy(s_be + (size_t)q * 2 * nk, s_be + (size_t)(q + 1) * 2 * nk,
                          beh.begin() + (size_t)q * ldbe + 2 * (k0 + 1));
                std::copy(s_rn + (size_t)q * nk, s_rn + (size_t)(q + 1) * nk, rnh.begin() + (size_t)q * ldrn + k0);
                flh[q] = s_fl[q];
            }
            bool newly = false;
            for (int q = 0; q < np; ++q) {
                BlPoint &p = pt[q];
                if (p.done) continue;
                const double b1r = beh[(size_t)q * ldbe], b1i = beh[(size_t)q * ldbe + 1];
                const double b1sr = b1r * b1r - b1i * b1i, b1si = 2.0 * b1r * b1i;   // beta_1^2
                const int brk = flh[q] >= 2 ? flh[q] - 2 : -1;                        // breakdown after this step
                for (int j = k0; j <= k && !p.done; ++j) {
                    const double ar = alh[(size_t)q * ldal + 2 * j], ai = alh[(size_t)q * ldal + 2 * j + 1];
                    double dr, di, zr, zi;
                    if (j == 0) {
                        dr = ar, di = ai, zr = 1.0, zi = 0.0;
                    } else {
                        const double br = beh[(size_t)q * ldbe + 2 * j], bi = beh[(size_t)q * ldbe + 2 * j + 1];
                        const double den = p.d_r * p.d_r + p.d_i * p.d_i;
                        const double lr = (br * p.d_r + bi * p.d_i) / den, li = (bi * p.d_r - br * p.d_i) / den;
                        dr = ar - (br * lr - bi * li);
                        di = ai - (br * li + bi * lr);
                        zr = -(lr * p.z_r - li * p.z_i);
                        zi = -(lr * p.z_i + li * p.z_r);
                    }
                    // P += beta_1^2 z^2 / d
                    const double z2r = zr * zr - zi * zi, z2i = 2.0 * zr * zi;
                    const double dd = dr * dr + di * di;
                    const double qr = (z2r * dr + z2i * di) / dd, qi = (z2i * dr - z2r * di) / dd;
                    p.P_r += b1sr * qr - b1si * qi;
                    p.P_i += b1sr * qi + b1si * qr;
                    p.d_r = dr, p.d_i = di, p.z_r = zr, p.z_i = zi;
                    p.steps = j + 1;
                    // |beta_1 z / d| |r| / |b|
                    const double res = std::sqrt((b1r * b1r + b1i * b1i) * (zr * zr + zi * zi) / dd) *
                                       rnh[(size_t)q * ldrn + j] / bnh[q];
                    const bool bad = !(dd > 0.0) || !std::isfinite(p.P_r) || !std::isfinite(p.P_i);
                    if (!bad && res <= tol) {
                        p.done = true, p.status = 0;
                    } else if (bad || j == brk) {
                        p.done = true, p.status = 2;
                    }
                }
                if (p.done) {
                    newly = true;
                    --active;
                    if (flh[q] == 0) flh[q] = 1;
                }
            }
            if (newly && active > 0) {
                std::copy(flh.begin(), flh.begin() + np, s_fl);
                HIPCHK(c, hipMemcpyAsync(flag, s_fl, (size_t)np * sizeof(int), hipMemcpyHostToDevice, s));
            }
            k0 = k + 1;
        }
        for (int q = 0; q < np; ++q) {
            const BlPoint &p = pt[q];
            const int64_t g = p0 + q;
            alpha[2 * g] = -p.P_r;
            alpha[2 * g + 1] = -p.P_i;
            if (steps) steps[g] = p.steps;
            const int st_q = p.done ? p.status : 1;
            if (status) status[g] = st_q;
            if (st_q != 0) rc = CHI0_NOT_CONVERGED;
        }
    }
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipGetLastError());
    return rc;
}
