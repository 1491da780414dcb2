// C ABI of libpat: problem handles, the forward and transpose maps, and the
// batched CGLS/RTO sampler.  Device work is enqueued on the caller's stream;
// each N_T-step sweep is captured once into a hipGraph and replayed.
//
// Paper: "3D Uncertainty Quantification for Photoacoustic Tomography"
// (arXiv 2607.21373): forward map Sec. 3 eq. (discrete-wave-matrix); transpose
// Sec. 5.1; extended least-squares problem Sec. 5 eq. (extended-matrices);
// RTO sample Algorithm 1; statistics Sec. 6.2 eq. (ergodic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pat_internal.h"
#include "pat_kernels.h"

namespace {

thread_local std::string g_err;

pat_status fail(pat_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define PAT_HIP(call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            (void)hipGetLastError();                                                                \
            return fail(e_ == hipErrorOutOfMemory ? PAT_ERR_OUT_OF_MEMORY : PAT_ERR_HIP,            \
                        std::string(#call) + ": " + hipGetErrorString(e_));                         \
        }                                                                                           \
    } while (0)

#define PAT_TRY(expr)                   \
    do {                                \
        pat_status s_ = (expr);         \
        if (s_ != PAT_OK) return s_;    \
    } while (0)

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
    int old = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) return;
        ok = (old == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

int choose_rb(int64_t R) {
    int rb = 1;
    while (rb < R && rb < 64) rb <<= 1;
    return rb;
}

// an explicit RHS block: a power of two up to the step kernels' limit for the sweep precision
bool valid_rb(int rb, pat::Prec pr) { return rb >= 1 && rb <= pat::max_rhs_block(pr) && (rb & (rb - 1)) == 0; }

size_t tsize(pat::Prec p) { return p == pat::Prec::F64 ? 8 : 4; }

// The vector-lane step kernels (rows of >= 16 bytes) address one block's state
// (N x block x element size) with 32-bit byte offsets, so it must stay below 4 GiB;
// the scalar-lane kernels use 64-bit indices.
bool block_fits(int64_t n, pat::Prec pr, int rb) {
    const uint64_t row = uint64_t(rb) * tsize(pr);
    return row < 16 || uint64_t(n) * row < (uint64_t(1) << 32);
}

// the largest block <= rb (halving) whose state fits the step kernels' addressing
int fit_rb(int64_t n, pat::Prec pr, int rb) {
    while (rb > 1 && !block_fits(n, pr, rb)) rb >>= 1;
    return rb;
}

pat_status check_block(int64_t n, pat::Prec pr, int rb) {
    if (block_fits(n, pr, rb)) return PAT_OK;
    return fail(PAT_ERR_INVALID_ARG, "RHS block of " + std::to_string(rb) + " too large for a mesh of " +
                                         std::to_string(n) + " nodes: one block's state must stay below 4 GiB");
}

}  // namespace

// Device scratch of pat_forward_noalloc, for callers that cannot allocate: one RHS
// block's sweep state (three rotating state vectors) and its data staging.  Each
// device holds its own copy from the library's first use on it until the process
// ends.  Host code
// never passes `scratch` itself to a kernel (on the host it only names the
// symbol): pat_problem_create looks up each device's copy with
// hipGetSymbolAddress and the entry point uses that address.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device ordinal -> address of its copy of `scratch`

// Look up the current device's copy of `scratch` once (the device must be current).
pat_status scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PAT_ERR_INVALID_ARG, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return PAT_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(PAT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
    return PAT_OK;
}

}  // namespace

struct SweepWS {
    pat::Prec prec = pat::Prec::F64;
    int RB = 0;
    // state buffers of the three-level steps: S[0] holds a forward sweep's input and
    // receives a transpose sweep's result
    void *S[3] = {nullptr, nullptr, nullptr};
    void *Y = nullptr;  // [M][RB] staging of the user-facing calls
    hipGraphExec_t g_fwd_user = nullptr, g_adj_user = nullptr;
    hipGraphExec_t g_fwd_cgls = nullptr, g_adj_cgls = nullptr;
    double g_fwd_cgls_scale = 0.0;
    const void *g_fwd_cgls_out = nullptr, *g_adj_cgls_in = nullptr;
    // float64 forward sweep of the final residual check (float64 workspaces only)
    hipGraphExec_t g_fwd_chk = nullptr;
    double g_fwd_chk_scale = 0.0;
    const void *g_fwd_chk_out = nullptr;
};

// Work buffers of the spectral prior for one RHS block.
struct SpecWS {
    double *gr = nullptr, *gc = nullptr;  // real and complex grid vectors [G][RB]
    double *ym = nullptr, *lx = nullptr;  // mesh [N][RB] and latent [G][RB] staging (float64)
};

struct CglsWS {
    int RB = 0;
    int cap_iter = -1;
    double *x = nullptr, *d = nullptr, *s = nullptr, *rp = nullptr, *qp = nullptr;
    double *rd = nullptr, *qd = nullptr, *Q = nullptr;
    double *part = nullptr, *mpart = nullptr, *coef = nullptr, *scal = nullptr;
    double *cg = nullptr, *gram = nullptr;  // reorthogonalisation: coefficients and Gram row, Gram matrix
    // LSQR: right vector v; z = G_ext w and the residual r = b - G_ext x, kept only for the histories
    double *v = nullptr, *zp = nullptr, *zd = nullptr, *lrp = nullptr, *lrd = nullptr;
};

struct pat_problem {
    int device = 0;
    pat::DevOps ops;
    pat_problem_info info{};
    bool perm_identity = true;
    std::vector<void *> allocs;
    std::vector<size_t> alloc_bytes;  // size of allocs[k]
    std::map<std::pair<int, int>, SweepWS> sweeps;
    std::map<std::pair<int, int64_t>, CglsWS> cgls;  // by (RB, unknowns per RHS)
    hipStream_t cap = nullptr;
    int64_t bytes = 0;
    // sweep timing
    bool prof = false;
    pat_profile prof_acc{};
    std::vector<hipEvent_t> events;
    // autotuned RHS block per (sample count, sweep precision)
    std::map<std::pair<int64_t, int>, int> tuned;
    // node coordinates in internal order [N][3] (for the spectral prior's interpolation)
    std::vector<double> xyz;
    // Whittle-Matern spectral prior (pat_spectral_prior_set)
    bool spec = false;
    pat_spectral_desc spec_desc{};
    pat::SpecOps sops;
    std::vector<void *> spec_allocs;
    std::map<int, SpecWS> specws;
};

// Several problems whose sweeps share launches (rto_sample_batch).
struct pat_batch {
    int device = 0;
    std::vector<pat_problem *> probs;
    hipStream_t cap = nullptr;
    hipGraphExec_t g_fwd = nullptr, g_adj = nullptr;
    std::vector<const void *> key_fwd, key_adj;
    std::vector<double> key_scale;
    bool key_mf = true, key_ma = true;
    // launch mode per direction (pat_batch_merge): 0 one launch per problem within each step,
    // 1 one merged launch per step, 2 each problem's whole sweep in turn; -1 tuned
    int force_mf = -1, force_ma = -1;
    // autotuned (RHS block, forward mode, transpose mode) per (S, precision)
    struct Tune {
        int rb;
        int mf, ma;
    };
    std::map<std::pair<int64_t, int>, Tune> tune;
};

namespace {

pat_status dev_alloc(pat_problem *p, void **ptr, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return fail(e == hipErrorOutOfMemory ? PAT_ERR_OUT_OF_MEMORY : PAT_ERR_HIP,
                    "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    p->allocs.push_back(*ptr);
    p->alloc_bytes.push_back(bytes);
    p->bytes += int64_t(bytes);
    return PAT_OK;
}

void dev_free(pat_problem *p, void *ptr) {
    if (!ptr) return;
    for (size_t k = 0; k < p->allocs.size(); ++k)
        if (p->allocs[k] == ptr) {
            p->allocs[k] = nullptr;
            p->bytes -= int64_t(p->alloc_bytes[k]);
        }
    (void)hipFree(ptr);
}

template <typename T>
pat_status upload(pat_problem *p, const std::vector<T> &h, const T **out) {
    void *d = nullptr;
    PAT_TRY(dev_alloc(p, &d, h.size() * sizeof(T)));
    if (!h.empty()) PAT_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<const T *>(d);
    return PAT_OK;
}

std::vector<float> to_f32(const std::vector<double> &v) {
    std::vector<float> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i]);
    return o;
}

pat_status get_sweep(pat_problem *p, pat::Prec prec, int RB, bool need_y, SweepWS **out) {
    SweepWS &w = p->sweeps[{int(prec), RB}];
    if (w.RB == 0) {
        // all three state buffers or none (a failed allocation leaves the workspace empty)
        const size_t bytes = size_t(p->ops.n) * RB * tsize(prec);
        void *v[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < 3; ++k) {
            pat_status st = dev_alloc(p, &v[k], bytes);
            if (st != PAT_OK) {
                for (int q = 0; q < k; ++q) dev_free(p, v[q]);
                return st;
            }
        }
        for (int k = 0; k < 3; ++k) w.S[k] = v[k];
        w.prec = prec;
        w.RB = RB;
    }
    if (need_y && !w.Y) {
        PAT_TRY(dev_alloc(p, &w.Y, size_t(p->ops.n_steps) * p->ops.n_obs * RB * tsize(prec)));
    }
    *out = &w;
    return PAT_OK;
}

// Capture the launches of one sweep on a capture stream.
template <class F>
pat_status capture_on(hipStream_t cap, hipGraphExec_t *exec, F &&body) {
    if (*exec) {
        (void)hipGraphExecDestroy(*exec);
        *exec = nullptr;
    }
    PAT_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    body(cap);
    hipGraph_t g = nullptr;
    PAT_HIP(hipStreamEndCapture(cap, &g));
    hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PAT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return PAT_OK;
}

template <class F>
pat_status capture(pat_problem *p, hipGraphExec_t *exec, F &&body) {
    return capture_on(p->cap, exec, std::forward<F>(body));
}

// Forward sweep: input state in w.S[0]; y^n (n = 1..N_T) written to y_out [N_T][N_obs][RB].
// Step k computes S^{k+1} from S^k and S^{k-1}, S^k in w.S[k % 3] (S^{-1} = S^0), and
// samples y^k of the state it reads.
void enqueue_forward(pat_problem *p, SweepWS &w, void *y_out, bool y_f64, double yscale, hipStream_t s) {
    const pat::DevOps &op = p->ops;
    const int NT = op.n_steps;
    for (int k = 0; k < NT; ++k)
        pat::launch_fwd_step(w.prec, w.RB, op, w.S[k % 3], w.S[k == 0 ? 0 : (k - 1) % 3], w.S[(k + 1) % 3], true,
                             k > 0, k - 1, y_out, y_f64, yscale, s);
    pat::launch_fwd_step(w.prec, w.RB, op, w.S[NT % 3], w.S[(NT - 1) % 3], nullptr, false, true, NT - 1, y_out,
                         y_f64, yscale, s);
}

// Buffer of q_j (j >= -1) in a transpose sweep of NT steps: chosen so that the
// result, written where q_{NT} would go, lands in S[0].
inline int adj_slot(int j, int NT) { return ((j - NT) % 3 + 3) % 3; }

// Transpose sweep: data yhat [N_T][N_obs][RB]; result G^T yhat in w.S[0].
void enqueue_adjoint(pat_problem *p, SweepWS &w, const void *yhat, bool y_f64, hipStream_t s) {
    const pat::DevOps &op = p->ops;
    const int NT = op.n_steps;
    auto q = [&](int j) { return w.S[adj_slot(j, NT)]; };
    pat::launch_adj_init(w.prec, w.RB, op, q(0), q(-1), yhat, y_f64, 1.0, s);
    for (int k = 0; k + 1 < NT; ++k)
        pat::launch_adj_step(w.prec, w.RB, op, q(k), q(k - 1), q(k + 1), false, NT - 2 - k, yhat, y_f64, 1.0, s);
    pat::launch_adj_step(w.prec, w.RB, op, q(NT - 1), q(NT - 2), q(NT), true, 0, yhat, y_f64, 1.0, s);
}

// Launch a sweep graph; with profiling on, bracket it with two events from the pool.
pat_status launch_sweep(pat_problem *p, hipGraphExec_t g, hipStream_t s, size_t *ev_used) {
    if (p->prof) {
        while (p->events.size() < *ev_used + 2) {
            hipEvent_t e;
            PAT_HIP(hipEventCreate(&e));
            p->events.push_back(e);
        }
        PAT_HIP(hipEventRecord(p->events[*ev_used], s));
        PAT_HIP(hipGraphLaunch(g, s));
        PAT_HIP(hipEventRecord(p->events[*ev_used + 1], s));
        *ev_used += 2;
        return PAT_OK;
    }
    PAT_HIP(hipGraphLaunch(g, s));
    return PAT_OK;
}

pat_status check_prec(pat_precision prec, pat::Prec *out) {
    if (prec == PAT_F64) *out = pat::Prec::F64;
    else if (prec == PAT_F32) *out = pat::Prec::F32;
    else return fail(PAT_ERR_INVALID_ARG, "precision must be PAT_F64 or PAT_F32");
    return PAT_OK;
}

// Solver workspace for RB right-hand sides with NX unknowns each (N, or n^3 in the
// latent space of the spectral prior).
pat_status get_cgls(pat_problem *p, int RB, int64_t NX, int n_iter, bool reorth, bool lsqr, bool track,
                    CglsWS **out) {
    CglsWS &c = p->cgls[{RB, NX}];
    const int64_t N = NX, M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    // each group of buffers is committed to the workspace only once all of it is allocated,
    // so a failed allocation never leaves a half-filled workspace behind
    auto alloc_group = [&](std::initializer_list<std::pair<double **, size_t>> group) -> pat_status {
        std::vector<void *> got;
        for (const auto &g : group) {
            void *v = nullptr;
            pat_status st = dev_alloc(p, &v, g.second);
            if (st != PAT_OK) {
                for (void *q : got) dev_free(p, q);
                return st;
            }
            got.push_back(v);
        }
        size_t k = 0;
        for (const auto &g : group) *g.first = static_cast<double *>(got[k++]);
        return PAT_OK;
    };
    const size_t nb = size_t(N) * RB * 8, mb = size_t(M) * RB * 8;
    if (c.RB == 0) {
        PAT_TRY(alloc_group({{&c.x, nb}, {&c.d, nb}, {&c.s, nb}, {&c.rp, nb}, {&c.qp, nb}, {&c.rd, mb},
                             {&c.qd, mb}, {&c.part, size_t(4) * pat::kDotBlocks * RB * 8},
                             {&c.scal, size_t(16) * RB * 8}}));
        c.RB = RB;
    }
    if (lsqr && !c.v) PAT_TRY(alloc_group({{&c.v, nb}}));
    if (lsqr && track && !c.zd) PAT_TRY(alloc_group({{&c.zp, nb}, {&c.lrp, nb}, {&c.lrd, mb}, {&c.zd, mb}}));
    const int need = reorth ? n_iter + 1 : 0;
    if (need > c.cap_iter) {
        dev_free(p, c.Q); dev_free(p, c.mpart); dev_free(p, c.coef); dev_free(p, c.cg); dev_free(p, c.gram);
        c.Q = c.mpart = c.coef = c.cg = c.gram = nullptr;
        c.cap_iter = 0;
        PAT_TRY(alloc_group({{&c.Q, size_t(need) * nb}, {&c.mpart, size_t(2 * need) * pat::kMultiBlocks * RB * 8},
                             {&c.coef, size_t(need) * RB * 8}, {&c.cg, size_t(2 * need) * RB * 8},
                             {&c.gram, size_t(need) * need * RB * 8}}));
        c.cap_iter = need;
    }
    *out = &c;
    return PAT_OK;
}


pat_status get_spec(pat_problem *p, int RB, SpecWS **out) {
    SpecWS &w = p->specws[RB];
    if (!w.gr) {
        const size_t G = size_t(p->sops.G), N = size_t(p->ops.n);
        const size_t sizes[4] = {G * RB * 8, G * RB * 16, N * RB * 8, G * RB * 8};
        void *v[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int k = 0; k < 4; ++k) {
            pat_status st = dev_alloc(p, &v[k], sizes[k]);
            if (st != PAT_OK) {
                for (int q = 0; q < k; ++q) dev_free(p, v[q]);
                return st;
            }
        }
        w.gc = static_cast<double *>(v[1]);
        w.ym = static_cast<double *>(v[2]);
        w.lx = static_cast<double *>(v[3]);
        w.gr = static_cast<double *>(v[0]);  // set last: marks the workspace complete
    }
    *out = &w;
    return PAT_OK;
}

// Free one sweep workspace and its graphs (the device is idle for it: callers
// synchronise first).
void release_sweep(pat_problem *p, pat::Prec prec, int RB) {
    auto it = p->sweeps.find({int(prec), RB});
    if (it == p->sweeps.end()) return;
    SweepWS &w = it->second;
    hipGraphExec_t *gs[] = {&w.g_fwd_user, &w.g_adj_user, &w.g_fwd_cgls, &w.g_adj_cgls, &w.g_fwd_chk};
    for (auto *g : gs)
        if (*g) (void)hipGraphExecDestroy(*g);
    void *bufs[] = {w.S[0], w.S[1], w.S[2], w.Y};
    for (void *b : bufs) dev_free(p, b);
    p->sweeps.erase(it);
}

// Sweep workspaces the autotuner creates for the candidate blocks it does not
// choose are released again; those that existed before it ran are kept.
struct TuneScope {
    std::vector<pat_problem *> probs;
    pat::Prec prec;
    std::vector<std::vector<int>> had;
    TuneScope(const std::vector<pat_problem *> &P, pat::Prec pr) : probs(P), prec(pr), had(P.size()) {
        for (size_t m = 0; m < P.size(); ++m)
            for (auto &kv : P[m]->sweeps)
                if (kv.first.first == int(pr)) had[m].push_back(kv.first.second);
    }
    void release_except(int keep) {
        for (size_t m = 0; m < probs.size(); ++m) {
            std::vector<int> made;
            for (auto &kv : probs[m]->sweeps)
                if (kv.first.first == int(prec) && kv.first.second != keep &&
                    std::find(had[m].begin(), had[m].end(), kv.first.second) == had[m].end())
                    made.push_back(kv.first.second);
            for (int rb : made) release_sweep(probs[m], prec, rb);
        }
    }
};

int auto_rb(const std::map<std::pair<int64_t, int>, int> &tuned, int64_t n, int64_t S, pat::Prec pr) {
    auto it = tuned.find({S, int(pr)});
    return it != tuned.end() ? it->second : fit_rb(n, pr, choose_rb(S));
}

// ---- several meshes per sweep launch ------------------------------------

// One launch per time step for all meshes (merge, vector-lane RHS blocks), else one per mesh.
void fwd_steps(pat::Prec prec, int RB, bool y_f64, const std::vector<pat::FwdStep> &st, hipStream_t s,
               bool merge = true) {
    if (merge && pat::multi_step_supported(prec, RB)) {
        pat::launch_fwd_multi(prec, RB, y_f64, st.data(), int(st.size()), s);
        return;
    }
    for (const pat::FwdStep &f : st)
        pat::launch_fwd_step(prec, RB, *f.op, f.S, f.Sp, f.Sn, f.rows, f.sample, f.t, f.y, y_f64,
                             f.yscale, s);
}

void adj_steps(pat::Prec prec, int RB, bool y_f64, const std::vector<pat::AdjStep> &st, hipStream_t s,
               bool merge = true) {
    if (merge && pat::multi_step_supported(prec, RB)) {
        pat::launch_adj_multi(prec, RB, y_f64, st.data(), int(st.size()), s);
        return;
    }
    for (const pat::AdjStep &a : st)
        pat::launch_adj_step(prec, RB, *a.op, a.S, a.Sp, a.Sn, a.last, a.tb, a.yh, y_f64, a.yscale, s);
}

// enqueue_forward for several meshes with equal N_T: the same launches, merged per step.
void enqueue_forward_multi(const std::vector<pat_problem *> &P, const std::vector<SweepWS *> &W,
                           const std::vector<void *> &yout, bool y_f64, const std::vector<double> &scale,
                           hipStream_t s, bool merge) {
    const size_t n = P.size();
    const int NT = P[0]->ops.n_steps;
    const pat::Prec prec = W[0]->prec;
    const int RB = W[0]->RB;
    std::vector<pat::FwdStep> st(n);
    for (int k = 0; k < NT; ++k) {
        for (size_t m = 0; m < n; ++m)
            st[m] = pat::FwdStep{&P[m]->ops, W[m]->S[k % 3], W[m]->S[k == 0 ? 0 : (k - 1) % 3], W[m]->S[(k + 1) % 3],
                                 true, k > 0, k - 1, yout[m], scale[m]};
        fwd_steps(prec, RB, y_f64, st, s, merge);
    }
    for (size_t m = 0; m < n; ++m)
        st[m] = pat::FwdStep{&P[m]->ops, W[m]->S[NT % 3], W[m]->S[(NT - 1) % 3], nullptr, false, true, NT - 1,
                             yout[m], scale[m]};
    fwd_steps(prec, RB, y_f64, st, s, merge);
}

// enqueue_adjoint for several meshes with equal N_T.
void enqueue_adjoint_multi(const std::vector<pat_problem *> &P, const std::vector<SweepWS *> &W,
                           const std::vector<const void *> &yin, bool y_f64, hipStream_t s, bool merge) {
    const size_t n = P.size();
    const int NT = P[0]->ops.n_steps;
    const pat::Prec prec = W[0]->prec;
    const int RB = W[0]->RB;
    auto q = [&](size_t m, int j) { return W[m]->S[adj_slot(j, NT)]; };
    for (size_t m = 0; m < n; ++m) pat::launch_adj_init(prec, RB, P[m]->ops, q(m, 0), q(m, -1), yin[m], y_f64, 1.0, s);
    std::vector<pat::AdjStep> st(n);
    for (int k = 0; k + 1 < NT; ++k) {
        for (size_t m = 0; m < n; ++m)
            st[m] = pat::AdjStep{&P[m]->ops, q(m, k), q(m, k - 1), q(m, k + 1), false, NT - 2 - k, yin[m], 1.0};
        adj_steps(prec, RB, y_f64, st, s, merge);
    }
    for (size_t m = 0; m < n; ++m)
        st[m] = pat::AdjStep{&P[m]->ops, q(m, NT - 1), q(m, NT - 2), q(m, NT), true, 0, yin[m], 1.0};
    adj_steps(prec, RB, y_f64, st, s, merge);
}

// Autotuner: for each candidate RHS block, time `reps` forward and transpose
// steps of all meshes (after a warm-up) with HIP events and price a run of S
// samples as ceil(S/RB) * (forward + transpose step); return the cheapest.  With
// several meshes each direction is timed merged (one launch per step) and one
// launch per mesh, and the faster is kept (*mf, *ma).
pat_status tune_rb(const std::vector<pat_problem *> &P, hipStream_t cap, int64_t S, pat::Prec pr, hipStream_t s,
                   int *best, double *best_us, int *mf = nullptr, int *ma = nullptr) {
    // candidates: up to the smallest block holding all S samples (beyond 64 only when S needs it)
    int top = 1;
    while (top < S && top < pat::max_rhs_block(pr)) top <<= 1;
    int64_t nmax = 0;
    for (const pat_problem *q : P) nmax = std::max<int64_t>(nmax, q->ops.n);
    top = fit_rb(nmax, pr, top);
    const int lo = std::max(1, std::min(top, 64) / 16);
    const int reps = 8;
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(PAT_ERR_HIP, "autotune: hipEventCreate failed");
        }
    *best = top;
    *best_us = 1e300;
    if (mf) *mf = 1;
    if (ma) *ma = 1;
    pat_status st = PAT_OK;
    for (int RB = lo; RB <= top && st == PAT_OK; RB <<= 1) {
        std::vector<SweepWS *> W(P.size());
        std::vector<void *> Y(P.size());
        std::vector<double> one(P.size(), 1.0);
        for (size_t m = 0; m < P.size() && st == PAT_OK; ++m) {
            st = get_sweep(P[m], pr, RB, true, &W[m]);
            if (st != PAT_OK) break;
            const size_t nb = size_t(P[m]->ops.n) * RB * tsize(pr);
            const size_t yb = size_t(P[m]->ops.n_steps) * P[m]->ops.n_obs * RB * tsize(pr);
            for (int k = 0; k < 3; ++k) {
                if (hipMemsetAsync(W[m]->S[k], 0, nb, s) != hipSuccess)
                    st = fail(PAT_ERR_HIP, "autotune: hipMemsetAsync failed");
            }
            if (hipMemsetAsync(W[m]->Y, 0, yb, s) != hipSuccess) st = fail(PAT_ERR_HIP, "autotune: hipMemsetAsync failed");
            Y[m] = W[m]->Y;
        }
        if (st != PAT_OK) break;
        const bool yf = pr == pat::Prec::F64;
        std::vector<pat::FwdStep> fs(P.size());
        std::vector<pat::AdjStep> as(P.size());
        for (size_t m = 0; m < P.size(); ++m) {
            fs[m] = pat::FwdStep{&P[m]->ops, W[m]->S[0], W[m]->S[1], W[m]->S[2], true, true, 0, Y[m], 1.0};
            // a plain step reads the data of sample times 0 and 1; one-step problems time the closing launch
            as[m] = pat::AdjStep{&P[m]->ops, W[m]->S[0], W[m]->S[1], W[m]->S[2], P[m]->ops.n_steps < 2, 0, Y[m], 1.0};
        }
        // The sweeps replay captured graphs, so time captured sequences of `reps` steps
        // (sequence q: direction q % 2).  Several meshes: q = 0, 1 merged launches per
        // step; q = 2, 3 one launch per mesh within each step; then one graph per mesh
        // and direction (that mesh alone, as a whole sweep per mesh runs it).
        const size_t nm = P.size();
        const bool multi = nm > 1;
        const int nq = multi ? 4 + 2 * int(nm) : 2;
        std::vector<hipGraphExec_t> g(size_t(nq), nullptr);
        for (int q = 0; q < nq && st == PAT_OK; ++q)
            st = capture_on(cap, &g[size_t(q)], [&](hipStream_t cs) {
                for (int k = 0; k < reps; ++k) {
                    if (q < 4) {
                        if (q % 2 == 0) fwd_steps(pr, RB, yf, fs, cs, q < 2);
                        else adj_steps(pr, RB, yf, as, cs, q < 2);
                    } else {
                        const size_t m = size_t(q - 4) / 2;
                        if (q % 2 == 0) fwd_steps(pr, RB, yf, {fs[m]}, cs, false);
                        else adj_steps(pr, RB, yf, {as[m]}, cs, false);
                    }
                }
            });
        std::vector<float> ms(size_t(nq), 0.f);
        if (st == PAT_OK) {
            for (int q = 0; q < nq && st == PAT_OK; ++q) {
                (void)hipGraphLaunch(g[size_t(q)], s);  // warm-up
                (void)hipEventRecord(ev[0], s);
                (void)hipGraphLaunch(g[size_t(q)], s);
                (void)hipEventRecord(ev[1], s);
                if (hipEventSynchronize(ev[1]) != hipSuccess) st = fail(PAT_ERR_HIP, "autotune: a timed step failed");
                else (void)hipEventElapsedTime(&ms[size_t(q)], ev[0], ev[1]);
            }
        }
        for (auto &x : g)
            if (x) (void)hipGraphExecDestroy(x);
        if (st != PAT_OK) break;
        float f_ms = ms[0], a_ms = ms[1];
        int m_f = 1, m_a = 1;
        if (multi) {
            const bool merged_ok = pat::multi_step_supported(pr, RB);
            if (!merged_ok || ms[2] < f_ms) { f_ms = ms[2]; m_f = 0; }
            if (!merged_ok || ms[3] < a_ms) { a_ms = ms[3]; m_a = 0; }
            float sf = 0.f, sa = 0.f;
            for (size_t m = 0; m < nm; ++m) {
                sf += ms[4 + 2 * m];
                sa += ms[5 + 2 * m];
            }
            if (sf < f_ms) { f_ms = sf; m_f = 2; }
            if (sa < a_ms) { a_ms = sa; m_a = 2; }
        }
        const double us = double((S + RB - 1) / RB) * 1e3 * double(f_ms + a_ms) / reps;
        if (us < *best_us) {
            *best_us = us;
            *best = RB;
            if (mf) *mf = m_f;
            if (ma) *ma = m_a;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (st == PAT_OK && hipGetLastError() != hipSuccess) st = fail(PAT_ERR_HIP, "autotune: launch failed");
    return st;
}

// One RHS block's least-squares solve, split into the phases between sweeps so
// that several blocks (of several meshes) can share each sweep launch:
//   init, [transpose sweep], post_adj(0),
//   then for k = 1..n_iter: pre_fwd(k), [forward sweep], post_fwd(k),
//   and unless k = n_iter: [transpose sweep], post_adj(k).
// The forward graph reads w->S[0] and writes qd = G x / sigma; the transpose
// graph reads rd and leaves G^T rd in w->S[0].
// With the spectral prior the unknowns are the latent grid vector (NX = n^3):
// G_ext = [G P / sigma ; I], the forward input is P x and the transpose output
// P^T (G^T r_d) / sigma + r_p.
struct Solve {
    pat_problem *p;
    SweepWS *w;
    CglsWS *c;
    pat::Prec pr;
    int RB, n_iter;
    bool reorth, lsqr;
    double isig, a;
    int64_t N, M, ld, S, rb0;
    double *resid_hist, *diag_hist;
    hipStream_t s;
    int64_t NX;       // unknowns per RHS
    SpecWS *sw;       // spectral prior work buffers, or null for the FE prior factor
};

// Residual history column `it` from the data part rd [M][RB] and prior part rp [N][RB].
void record(Solve &v, const double *rd, const double *rp, int it) {
    if (!v.resid_hist && !v.diag_hist) return;
    double *pA = v.c->part, *pB = v.c->part + pat::kDotBlocks * v.RB;
    double *t1 = v.c->scal + 14 * v.RB, *t2 = v.c->scal + 15 * v.RB;
    pat::launch_dot_partial(rd, rd, v.M, v.RB, pA, v.s);
    pat::launch_dot_partial(rp, rp, v.NX, v.RB, pB, v.s);
    pat::launch_dot_final(pA, nullptr, v.RB, t1, v.s);
    pat::launch_dot_final(pB, nullptr, v.RB, t2, v.s);
    pat::launch_resid(t1, t2, v.resid_hist, v.diag_hist, v.ld, it, v.rb0, v.S, v.RB, v.s);
}

// s -= Q coef over the basis Q_j, j < k: classical Gram-Schmidt applied twice, in the
// form that reads the basis twice instead of four times.  The first pass's
// coefficients c1 = Q^T s and the newest basis vector's row of the Gram matrix
// Q^T Q come from one read of Q; the second pass's coefficients follow from them,
// c2 = Q^T (s - Q c1) = c1 - (Q^T Q) c1; one projection s -= Q (c1 + c2) ends it.
// Equal to the two passes in exact arithmetic.
void reorthogonalise(Solve &v, int k) {
    if (!v.reorth || k <= 0) return;
    pat::launch_reorth_coef(v.c->Q, v.c->s, k, v.NX, v.RB, v.c->mpart, v.c->cg, v.c->gram, v.c->cap_iter, v.c->coef,
                            v.s);
    pat::launch_project(v.c->Q, v.c->s, v.c->coef, k, v.NX, v.RB, v.s);
}

// s = G^T rd / sigma + L^T up (spectral prior: P^T G^T rd / sigma + up), from the transpose sweep's result.
void combine_t(Solve &v, const double *up) {
    if (v.sw)
        pat::launch_spectral_t(v.p->sops, v.RB, v.w->S[0], v.pr, v.isig, up, v.sw->gr, v.sw->gc, v.c->s, v.s);
    else
        pat::launch_gext_t_combine(v.pr, v.p->ops, v.RB, v.a, v.isig, v.w->S[0], up, v.c->s, v.s);
}

// qp = L x (spectral prior: the identity on the latent vector).
void prior_part(Solve &v, const double *x) {
    if (v.sw) pat::launch_lincomb(v.c->qp, x, nullptr, 1.0, nullptr, nullptr, 0.0, v.NX, v.RB, v.s);
    else pat::launch_prior(v.p->ops, v.RB, v.a, x, v.c->qp, v.s);
}

// ---- CGLS: b in (rd, rp) and x = 0 on entry.  The normal-equation residuals
// s_j are kept orthogonal by two classical Gram-Schmidt passes (App. A).
struct CglsScal {
    double *gamma, *delta, *alpha, *beta, *invn, *gnew;
    explicit CglsScal(const Solve &v)
        : gamma(v.c->scal), delta(v.c->scal + v.RB), alpha(v.c->scal + 2 * v.RB), beta(v.c->scal + 3 * v.RB),
          invn(v.c->scal + 4 * v.RB), gnew(v.c->scal + 5 * v.RB) {}
};

void cgls_post_adj(Solve &v, int k) {
    CglsWS *c = v.c;
    const CglsScal z(v);
    double *pA = c->part;
    combine_t(v, c->rp);
    reorthogonalise(v, k);
    pat::launch_dot_partial(c->s, c->s, v.NX, v.RB, pA, v.s);
    pat::launch_dot_final(pA, nullptr, v.RB, z.gnew, v.s);
    // beta = gamma_new / gamma ; d = s + beta d ; Q[k] = s / ||s||
    pat::launch_scalar_gamma(z.gamma, z.gnew, z.beta, z.invn, k == 0, v.RB, v.s);
    pat::launch_append_dir(c->s, v.reorth ? c->Q + size_t(k) * v.NX * v.RB : nullptr, c->d, z.invn, z.beta, k == 0,
                           v.NX, v.RB, v.s);
}

void cgls_post_fwd(Solve &v, int k) {
    CglsWS *c = v.c;
    const CglsScal z(v);
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * v.RB;
    // q = (G d / sigma, L d) ; alpha = gamma / ||q||^2 ; x += alpha d ; r -= alpha q
    prior_part(v, c->d);
    pat::launch_dot_partial(c->qd, c->qd, v.M, v.RB, pA, v.s);
    pat::launch_dot_partial(c->qp, c->qp, v.NX, v.RB, pB, v.s);
    pat::launch_dot_final(pA, pB, v.RB, z.delta, v.s);
    pat::launch_scalar_alpha(z.gamma, z.delta, z.alpha, v.RB, v.s);
    pat::launch_update_xr(c->x, c->d, c->rp, c->qp, z.alpha, v.NX, v.RB, v.s);
    pat::launch_axpy_neg(c->rd, c->qd, z.alpha, v.M, v.RB, v.s);
    record(v, c->rd, c->rp, k);
}

// ---- LSQR (Paige and Saunders' bidiagonalisation, the solver of Sec. 5 and Algorithm 1):
// b in (rd, rp) and x = 0 on entry.  The left vector u lives in (rd, rp), so
// the transpose graph reads it where CGLS keeps its residual; the search
// direction w lives in d.  The residual b - G_ext x is carried (through
// z = G_ext w) only when a history is asked for.
struct LsqrState {
    pat::LsqrScalars L;
    double *n1, *n2;
    bool track;
    explicit LsqrState(const Solve &v) {
        double *sc = v.c->scal;
        const int RB = v.RB;
        L = pat::LsqrScalars{sc, sc + RB, sc + 2 * RB, sc + 3 * RB, sc + 4 * RB, sc + 5 * RB,
                             sc + 6 * RB, sc + 7 * RB, sc + 8 * RB, sc + 9 * RB, sc + 10 * RB, sc + 11 * RB};
        n1 = sc + 12 * RB;
        n2 = sc + 13 * RB;
        track = v.resid_hist || v.diag_hist;
    }
};

void lsqr_init(Solve &v) {
    CglsWS *c = v.c;
    const LsqrState z(v);
    const int RB = v.RB;
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * RB;
    if (z.track) {
        pat::launch_lincomb(c->lrd, c->rd, nullptr, 1.0, nullptr, nullptr, 0.0, v.M, RB, v.s);
        pat::launch_lincomb(c->lrp, c->rp, nullptr, 1.0, nullptr, nullptr, 0.0, v.NX, RB, v.s);
        record(v, c->lrd, c->lrp, 0);
    }
    // beta_1 u_1 = b
    pat::launch_dot_partial(c->rd, c->rd, v.M, RB, pA, v.s);
    pat::launch_dot_partial(c->rp, c->rp, v.NX, RB, pB, v.s);
    pat::launch_dot_final(pA, nullptr, RB, z.n1, v.s);
    pat::launch_dot_final(pB, nullptr, RB, z.n2, v.s);
    pat::launch_lsqr_scalar(pat::LsqrStage::InitBeta, z.L, z.n1, z.n2, RB, v.s);
    pat::launch_lincomb(c->rd, c->rd, z.L.inv, 1.0, nullptr, nullptr, 0.0, v.M, RB, v.s);
    pat::launch_lincomb(c->rp, c->rp, z.L.inv, 1.0, nullptr, nullptr, 0.0, v.NX, RB, v.s);
}

void lsqr_post_adj(Solve &v, int k) {
    CglsWS *c = v.c;
    const LsqrState z(v);
    double *pA = c->part;
    // alpha_{k+1} v_{k+1} = G_ext^T u_{k+1} - beta_{k+1} v_k, reorthogonalised ; w = v - zfac w
    combine_t(v, c->rp);
    if (k > 0) pat::launch_lincomb(c->s, c->s, nullptr, 1.0, c->v, z.L.beta, -1.0, v.NX, v.RB, v.s);
    reorthogonalise(v, k);
    pat::launch_dot_partial(c->s, c->s, v.NX, v.RB, pA, v.s);
    pat::launch_dot_final(pA, nullptr, v.RB, z.n1, v.s);
    pat::launch_lsqr_scalar(k == 0 ? pat::LsqrStage::InitAlpha : pat::LsqrStage::Alpha, z.L, z.n1, nullptr, v.RB, v.s);
    pat::launch_lsqr_vw(c->s, z.L.inv, z.L.zfac, c->v, c->d, v.reorth ? c->Q + size_t(k) * v.NX * v.RB : nullptr,
                        k == 0, v.NX, v.RB, v.s);
}

void lsqr_post_fwd(Solve &v, int k) {
    CglsWS *c = v.c;
    const LsqrState z(v);
    const int RB = v.RB;
    const int64_t N = v.NX, M = v.M;
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * RB;
    // q = G_ext v_k ; z_k = q - zfac z_{k-1}
    prior_part(v, c->v);
    if (z.track) {
        pat::launch_lincomb(c->zd, c->qd, nullptr, 1.0, k > 1 ? c->zd : nullptr, z.L.zfac, -1.0, M, RB, v.s);
        pat::launch_lincomb(c->zp, c->qp, nullptr, 1.0, k > 1 ? c->zp : nullptr, z.L.zfac, -1.0, N, RB, v.s);
    }
    // beta_{k+1} u_{k+1} = q - alpha_k u_k ; plane rotation
    pat::launch_lincomb(c->rd, c->qd, nullptr, 1.0, c->rd, z.L.alpha, -1.0, M, RB, v.s);
    pat::launch_lincomb(c->rp, c->qp, nullptr, 1.0, c->rp, z.L.alpha, -1.0, N, RB, v.s);
    pat::launch_dot_partial(c->rd, c->rd, M, RB, pA, v.s);
    pat::launch_dot_partial(c->rp, c->rp, N, RB, pB, v.s);
    pat::launch_dot_final(pA, nullptr, RB, z.n1, v.s);
    pat::launch_dot_final(pB, nullptr, RB, z.n2, v.s);
    pat::launch_lsqr_scalar(pat::LsqrStage::Beta, z.L, z.n1, z.n2, RB, v.s);
    pat::launch_lincomb(c->rd, c->rd, z.L.inv, 1.0, nullptr, nullptr, 0.0, M, RB, v.s);
    pat::launch_lincomb(c->rp, c->rp, z.L.inv, 1.0, nullptr, nullptr, 0.0, N, RB, v.s);
    // x += (phi/rho) w ; r -= (phi/rho) z
    pat::launch_lincomb(c->x, c->x, nullptr, 1.0, c->d, z.L.step, 1.0, N, RB, v.s);
    if (z.track) {
        pat::launch_lincomb(c->lrd, c->lrd, nullptr, 1.0, c->zd, z.L.step, -1.0, M, RB, v.s);
        pat::launch_lincomb(c->lrp, c->lrp, nullptr, 1.0, c->zp, z.L.step, -1.0, N, RB, v.s);
        record(v, c->lrd, c->lrp, k);
    }
}

// ---- phase dispatch
void ph_init(Solve &v) {
    if (v.lsqr) lsqr_init(v);
    else record(v, v.c->rd, v.c->rp, 0);
}
void ph_post_adj(Solve &v, int k) { v.lsqr ? lsqr_post_adj(v, k) : cgls_post_adj(v, k); }
void ph_pre_fwd(Solve &v, int) {
    // the forward graph reads its input from S[0] in the sweep precision
    const double *x = v.lsqr ? v.c->v : v.c->d;
    if (v.sw) pat::launch_spectral(v.p->sops, v.RB, x, v.sw->gr, v.sw->gc, v.pr, v.w->S[0], v.N, v.s);
    else pat::launch_cast_to_state(v.pr, x, v.w->S[0], v.N * v.RB, v.s);
}
void ph_post_fwd(Solve &v, int k) { v.lsqr ? lsqr_post_fwd(v, k) : cgls_post_fwd(v, k); }
// per-RHS scalar that turns non-finite when the solve breaks down (CGLS gamma, LSQR phi_bar)
const double *ph_check(const Solve &v) { return v.lsqr ? v.c->scal + 5 * v.RB : v.c->scal; }

// Run the blocks in lockstep; fwd() and adj() launch one shared sweep each.
template <class Fwd, class Adj>
pat_status drive(std::vector<Solve> &blocks, int n_iter, Fwd &&fwd, Adj &&adj) {
    for (Solve &v : blocks) ph_init(v);
    PAT_TRY(adj());
    for (Solve &v : blocks) ph_post_adj(v, 0);
    for (int k = 1; k <= n_iter; ++k) {
        for (Solve &v : blocks) ph_pre_fwd(v, k);
        PAT_TRY(fwd());
        for (Solve &v : blocks) ph_post_fwd(v, k);
        if (k == n_iter) break;
        PAT_TRY(adj());
        for (Solve &v : blocks) ph_post_adj(v, k);
    }
    return PAT_OK;
}

// b = (y_obs/sigma + eta, xi) of block rb0 in (rd, rp), from the caller's draws or the device streams.
void build_b(Solve &v, const double *y_obs, const pat_rto_params *prm) {
    const pat::DevOps &op = v.p->ops;
    // latent grid vectors keep the caller's (grid) order
    const int32_t *perm = (v.sw || v.p->perm_identity) ? nullptr : op.perm;
    if (prm->eta) {
        pat::launch_build_rhs(y_obs, prm->eta, v.S, v.rb0, v.RB, v.M, v.isig, v.c->rd, v.s);
        pat::launch_pack(true, true, prm->xi, v.S, v.rb0, v.RB, v.NX, perm, v.c->rp, v.s);
    } else {
        pat::launch_build_rhs_rng(y_obs, prm->seed, prm->sample0, v.S, v.rb0, v.RB, v.M, v.isig, v.c->rd, v.s);
        pat::launch_xi_rng(prm->seed, prm->sample0, v.S, v.rb0, v.RB, v.NX, perm, v.c->rp, v.s);
    }
}

// b in (rd, rp) and the starting point x = 0 of block rb0.
void build_rhs(Solve &v, const double *y_obs, const pat_rto_params *prm) {
    build_b(v, y_obs, prm);
    pat::launch_fill(v.c->x, v.NX * v.RB, 0.0, v.s);
}

// Float64 check of a finished block: out[rb0 + r] = ||b - G_ext x||_2 of its samples
// (Sec. 5 eq. (lsqr-residual)), recomputed from x with a float64 forward sweep and the
// float64 prior factor whatever the solver's sweep precision, unlike the residual the
// solver carries.  rd, rp, qd and qp are free once the solve has ended, so b is rebuilt
// in (rd, rp).  Blocks wider than the float64 step kernels take (one float64 sweep per
// slice of at most 128 right-hand sides).
pat_status final_check(Solve &v, const double *y_obs, const pat_rto_params *prm, double *out) {
    if (!out) return PAT_OK;
    pat_problem *p = v.p;
    CglsWS *c = v.c;
    const int RB = v.RB;
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * RB;
    double *t1 = c->scal + 14 * RB, *t2 = c->scal + 15 * RB;
    build_b(v, y_obs, prm);
    prior_part(v, c->x);  // qp = L x (latent prior: x)
    pat::launch_lincomb(c->rp, c->rp, nullptr, 1.0, c->qp, nullptr, -1.0, v.NX, RB, v.s);
    pat::launch_dot_partial(c->rp, c->rp, v.NX, RB, pB, v.s);
    pat::launch_dot_final(pB, nullptr, RB, t2, v.s);
    const int RBf = fit_rb(v.N, pat::Prec::F64, std::min(RB, pat::max_rhs_block(pat::Prec::F64)));
    SweepWS *w64;
    PAT_TRY(get_sweep(p, pat::Prec::F64, RBf, false, &w64));
    if (!w64->g_fwd_chk || w64->g_fwd_chk_out != c->qd || w64->g_fwd_chk_scale != v.isig) {
        PAT_TRY(capture(p, &w64->g_fwd_chk, [&](hipStream_t cs) { enqueue_forward(p, *w64, c->qd, true, v.isig, cs); }));
        w64->g_fwd_chk_out = c->qd;
        w64->g_fwd_chk_scale = v.isig;
    }
    const double *src = c->x;
    if (v.sw) {  // the sample p0 = P w of the latent solution
        pat::launch_spectral(p->sops, RB, c->x, v.sw->gr, v.sw->gc, pat::Prec::F64, v.sw->ym, v.N, v.s);
        src = v.sw->ym;
    }
    for (int h = 0; h < RB; h += RBf) {
        pat::launch_cols(src, RB, h, static_cast<double *>(w64->S[0]), v.N, RBf, v.s);
        PAT_HIP(hipGraphLaunch(w64->g_fwd_chk, v.s));  // qd [M][RBf] = G p / sigma
        pat::launch_diff_sq_partial(c->rd, RB, h, c->qd, v.M, RBf, pA, v.s);
        pat::launch_dot_final(pA, nullptr, RBf, t1 + h, v.s);
    }
    pat::launch_resid(t1, t2, out, nullptr, 1, 0, v.rb0, v.S, RB, v.s);
    return PAT_OK;
}

// Samples of the finished block in the caller's layout: p0 = x (FE prior) or p0 = P x
// (spectral prior, whose latent x also goes to prm->latent when given).
void finish_block(Solve &v, const pat_rto_params *prm, double *samples) {
    const pat::DevOps &op = v.p->ops;
    const int32_t *perm = v.p->perm_identity ? nullptr : op.perm;
    if (v.sw) {
        pat::launch_spectral(v.p->sops, v.RB, v.c->x, v.sw->gr, v.sw->gc, pat::Prec::F64, v.sw->ym, v.N, v.s);
        pat::launch_unpack(true, true, v.sw->ym, v.S, v.rb0, v.RB, v.N, perm, samples, v.s);
        if (prm->latent) pat::launch_unpack(true, true, v.c->x, v.S, v.rb0, v.RB, v.NX, nullptr, prm->latent, v.s);
    } else {
        pat::launch_unpack(true, true, v.c->x, v.S, v.rb0, v.RB, v.N, perm, samples, v.s);
    }
}

// The solver state of block rb0 of problem p.
pat_status make_solve(pat_problem *p, const pat_rto_params *prm, pat::Prec pr, int RB, int64_t S, int64_t rb0,
                      double *resid_hist, hipStream_t s, Solve *out) {
    const bool spec = prm->prior == PAT_PRIOR_SPECTRAL;
    const bool reorth = prm->reorth != 0, lsqr = prm->solver == PAT_LSQR;
    const int64_t N = p->ops.n, M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    const int64_t NX = spec ? p->sops.G : N;
    SweepWS *w;
    PAT_TRY(get_sweep(p, pr, RB, false, &w));
    CglsWS *c;
    PAT_TRY(get_cgls(p, RB, NX, prm->n_iter, reorth, lsqr, resid_hist || prm->diag_hist, &c));
    SpecWS *sw = nullptr;
    if (spec) PAT_TRY(get_spec(p, RB, &sw));
    *out = Solve{p, w, c, pr, RB, prm->n_iter, reorth, lsqr, 1.0 / prm->sigma, prm->prior_a, N, M,
                 int64_t(prm->n_iter) + 1, S, rb0, resid_hist, prm->diag_hist, s, NX, sw};
    return PAT_OK;
}

pat_status check_rto_params(const pat_rto_params *prm, int64_t S, bool want_std) {
    if ((prm->eta == nullptr) != (prm->xi == nullptr))
        return fail(PAT_ERR_INVALID_ARG, "rto_sample: pass both eta and xi, or neither (device draws)");
    if (prm->sample0 < 0) return fail(PAT_ERR_INVALID_ARG, "rto_sample: sample0 must be >= 0");
    if (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma)) return fail(PAT_ERR_INVALID_ARG, "sigma must be > 0");
    if (!(prm->prior_a >= 0.0) || !std::isfinite(prm->prior_a)) return fail(PAT_ERR_INVALID_ARG, "prior_a must be >= 0");
    if (prm->n_iter < 1) return fail(PAT_ERR_INVALID_ARG, "n_iter must be >= 1");
    if (want_std && S < 2) return fail(PAT_ERR_INVALID_ARG, "std needs S >= 2");
    if (prm->rhs_block != 0 &&
        !valid_rb(prm->rhs_block, prm->sweep_prec == PAT_F64 ? pat::Prec::F64 : pat::Prec::F32))
        return fail(PAT_ERR_INVALID_ARG,
                    "rhs_block must be 0 or a power of two <= 256 (float32 sweeps) or <= 128 (float64 sweeps)");
    if (prm->solver != PAT_CGLS && prm->solver != PAT_LSQR)
        return fail(PAT_ERR_INVALID_ARG, "solver must be PAT_CGLS or PAT_LSQR");
    if (prm->prior != PAT_PRIOR_FE && prm->prior != PAT_PRIOR_SPECTRAL)
        return fail(PAT_ERR_INVALID_ARG, "prior must be PAT_PRIOR_FE or PAT_PRIOR_SPECTRAL");
    return PAT_OK;
}

pat_status check_spectral(const pat_problem *p, const pat_rto_params *prm, int RB) {
    if (prm->prior != PAT_PRIOR_SPECTRAL) return PAT_OK;
    if (!p->spec) return fail(PAT_ERR_INVALID_ARG, "spectral prior requested but none set (pat_spectral_prior_set)");
    if (!pat::spectral_rb_ok(RB)) return fail(PAT_ERR_INVALID_ARG, "rhs_block not supported by the spectral prior");
    return PAT_OK;
}

// Per-sweep event timings of the last call, folded into the handle's profile.
pat_status fold_profile(pat_problem *p, const std::vector<int> &ev_kind) {
    for (size_t q = 0; q < ev_kind.size(); ++q) {
        float ms = 0.f;
        PAT_HIP(hipEventElapsedTime(&ms, p->events[2 * q], p->events[2 * q + 1]));
        if (ev_kind[q] == 0) {
            p->prof_acc.fwd_ms += ms;
            ++p->prof_acc.fwd_sweeps;
        } else {
            p->prof_acc.adj_ms += ms;
            ++p->prof_acc.adj_sweeps;
        }
    }
    return PAT_OK;
}

// Capture (or reuse) a problem's solver sweep graphs for output scale isig.
pat_status solver_graphs(pat_problem *p, SweepWS *w, CglsWS *c, double isig) {
    if (!w->g_fwd_cgls || w->g_fwd_cgls_scale != isig || w->g_fwd_cgls_out != c->qd) {
        PAT_TRY(capture(p, &w->g_fwd_cgls, [&](hipStream_t cs) { enqueue_forward(p, *w, c->qd, true, isig, cs); }));
        w->g_fwd_cgls_scale = isig;
        w->g_fwd_cgls_out = c->qd;
    }
    if (!w->g_adj_cgls || w->g_adj_cgls_in != c->rd) {
        PAT_TRY(capture(p, &w->g_adj_cgls, [&](hipStream_t cs) { enqueue_adjoint(p, *w, c->rd, true, cs); }));
        w->g_adj_cgls_in = c->rd;
    }
    return PAT_OK;
}

}  // namespace

extern "C" {

const char *pat_last_error(void) { return g_err.c_str(); }

const char *pat_version(void) { return "libpat 0.1 (gfx950)"; }

pat_status pat_problem_create(const pat_problem_desc *desc, pat_problem **out) {
    g_err.clear();
    if (!desc || !out) return fail(PAT_ERR_INVALID_ARG, "NULL descriptor or output handle");
    *out = nullptr;
    // host validation and assembly first: no device work before the input is known good
    pat::HostProblem hp;
    std::string err;
    pat_status st = pat::build_host_problem(*desc, hp, err);
    if (st != PAT_OK) return fail(st, err);

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return fail(PAT_ERR_HIP, "no HIP device available");
    }
    int dev = desc->device;
    if (dev < 0) PAT_HIP(hipGetDevice(&dev));
    if (dev >= ndev) return fail(PAT_ERR_INVALID_ARG, "device ordinal out of range");
    DeviceGuard guard(dev);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");

    PAT_TRY(scratch_init(dev));
    auto p = std::make_unique<pat_problem>();
    p->device = dev;
    pat::DevOps &op = p->ops;
    op.n = hp.n;
    op.n_obs = hp.n_obs;
    op.n_steps = hp.n_steps;
    op.nnz = hp.rowptr.back();
    op.dt = hp.dt;

    std::vector<double> dtm(hp.n), sqm(hp.n), isqm(hp.n);
    for (int32_t i = 0; i < hp.n; ++i) {
        dtm[i] = hp.dt / hp.mass[i];
        sqm[i] = std::sqrt(hp.mass[i]);
        isqm[i] = 1.0 / sqm[i];
    }
    auto cleanup = [&](pat_status s) {
        for (void *a : p->allocs)
            if (a) (void)hipFree(a);
        p->allocs.clear();
        p->alloc_bytes.clear();
        return s;
    };
#define UP(vec, field)                                   \
    do {                                                 \
        pat_status s_ = upload(p.get(), vec, &op.field); \
        if (s_ != PAT_OK) return cleanup(s_);            \
    } while (0)
    UP(hp.rowptr, rowptr);
    UP(hp.col, col);
    UP(hp.snode, snode);
    UP(hp.injptr, injptr);
    UP(hp.injs, injs);
    UP(hp.perm, perm);
    UP(hp.k1val, k1val64);
    UP(dtm, dtm64);
    UP(sqm, sqrtm);
    UP(isqm, isqrtm);
    UP(hp.sw, sw64);
    UP(hp.injw, injw64);
    UP(to_f32(dtm), dtm32);
    UP(to_f32(hp.sw), sw32);
    UP(to_f32(hp.injw), injw32);
    UP(hp.ell_col, ell_col);
    UP(hp.xptr, xptr);
    UP(hp.xcol, xcol);
    UP(hp.bsoff, bsoff);
    UP(hp.bnum, bnum);
    UP(hp.ell_val, ell_val64);
    UP(hp.xval, xval64);
    UP(hp.bslot, bslot64);
    UP(to_f32(hp.ell_val), ell_val32);
    UP(to_f32(hp.xval), xval32);
    UP(to_f32(hp.bslot), bslot32);
    {
        pat::HaloTiles ht;
        pat::build_halo_tiles(hp, ht);
        UP(ht.desc, ht_desc);
        UP(ht.hrow, ht_hrow);
        UP(ht.meta, ht_meta);
        op.n_ht = ht.n_tiles;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return cleanup(fail(PAT_ERR_HIP, "hipDeviceGetAttribute failed"));
        op.n_cu = ncu;
    }
#undef UP
    p->perm_identity = true;
    for (int32_t i = 0; i < hp.n; ++i)
        if (hp.perm[i] != i) p->perm_identity = false;
    p->xyz.resize(size_t(hp.n) * 3);
    for (int32_t i = 0; i < hp.n; ++i)
        for (int d = 0; d < 3; ++d) p->xyz[size_t(i) * 3 + d] = desc->coords[size_t(hp.perm[i]) * 3 + d];
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(PAT_ERR_HIP, "hipStreamCreateWithFlags failed"));

    pat_problem_info &in = p->info;
    in.n_nodes = hp.n;
    in.n_obs = hp.n_obs;
    in.n_steps = hp.n_steps;
    in.n_tets = hp.n_tets;
    in.nnz_k = hp.rowptr.back();
    in.nnz_b = hp.nnz_b;
    in.n_boundary_nodes = hp.n_boundary;
    in.max_row_nnz = hp.max_row;
    in.dt = hp.dt;
    in.lambda_max = hp.lambda_max;
    in.b_stored = int64_t(hp.bval.size());
    *out = p.release();
    return PAT_OK;
}

pat_status pat_problem_destroy(pat_problem *p) {
    if (!p) return PAT_OK;
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : p->sweeps) {
        SweepWS &w = kv.second;
        hipGraphExec_t *gs[] = {&w.g_fwd_user, &w.g_adj_user, &w.g_fwd_cgls, &w.g_adj_cgls, &w.g_fwd_chk};
        for (auto *g : gs)
            if (*g) (void)hipGraphExecDestroy(*g);
    }
    for (void *a : p->allocs)
        if (a) (void)hipFree(a);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    delete p;
    return PAT_OK;
}

pat_status pat_problem_get_info(const pat_problem *p, pat_problem_info *out) {
    if (!p || !out) return fail(PAT_ERR_INVALID_ARG, "NULL handle or output");
    *out = p->info;
    out->device_bytes = p->bytes;
    return PAT_OK;
}

pat_status pat_forward(pat_problem *p, int64_t R, const void *p0, void *y, pat_precision prec, void *stream) {
    g_err.clear();
    if (!p || !p0 || !y || R < 1) return fail(PAT_ERR_INVALID_ARG, "pat_forward: NULL pointer or R < 1");
    pat::Prec pr;
    PAT_TRY(check_prec(prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int RB = fit_rb(p->ops.n, pr, choose_rb(R));
    PAT_TRY(check_block(p->ops.n, pr, RB));
    SweepWS *w;
    PAT_TRY(get_sweep(p, pr, RB, true, &w));
    if (!w->g_fwd_user)
        PAT_TRY(capture(p, &w->g_fwd_user, [&](hipStream_t cs) { enqueue_forward(p, *w, w->Y, false, 1.0, cs); }));
    const bool f64 = pr == pat::Prec::F64;
    const int64_t M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        pat::launch_pack(f64, f64, p0, R, rb0, RB, p->ops.n, perm, w->S[0], s);
        PAT_HIP(hipGraphLaunch(w->g_fwd_user, s));
        pat::launch_unpack(f64, f64, w->Y, R, rb0, RB, M, nullptr, y, s);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_forward_noalloc(pat_problem *p, int64_t R, const void *p0, void *y, pat_precision prec,
                               void *stream) {
    g_err.clear();
    if (!p || !p0 || !y || R < 1) return fail(PAT_ERR_INVALID_ARG, "pat_forward_noalloc: NULL pointer or R < 1");
    pat::Prec pr;
    PAT_TRY(check_prec(prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    char *base = static_cast<char *>(p->device < kMaxDevices ? g_scratch_ptr[p->device] : nullptr);
    if (!base) return fail(PAT_ERR_INTERNAL, "pat_forward_noalloc: no scratch address for the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    // the block of pat_forward, halved until three state vectors and the staging fit the scratch
    auto need = [&](int rb) { return 3 * up(size_t(p->ops.n) * rb * tsize(pr)) + up(size_t(M) * rb * tsize(pr)); };
    int RB = fit_rb(p->ops.n, pr, choose_rb(R));
    while (RB > 1 && need(RB) > kScratchBytes) RB >>= 1;
    if (need(RB) > kScratchBytes)
        return fail(PAT_ERR_INVALID_ARG, "pat_forward_noalloc: one right-hand side needs " + std::to_string(need(1)) +
                                             " bytes of scratch, more than its " + std::to_string(kScratchBytes));
    PAT_TRY(check_block(p->ops.n, pr, RB));
    SweepWS w;  // a view of the scratch: nothing is allocated
    w.prec = pr;
    w.RB = RB;
    const size_t nb = up(size_t(p->ops.n) * RB * tsize(pr));
    w.S[0] = base;
    w.S[1] = base + nb;
    w.S[2] = base + 2 * nb;
    w.Y = base + 3 * nb;
    const bool f64 = pr == pat::Prec::F64;
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        pat::launch_pack(f64, f64, p0, R, rb0, RB, p->ops.n, perm, w.S[0], s);
        enqueue_forward(p, w, w.Y, false, 1.0, s);
        pat::launch_unpack(f64, f64, w.Y, R, rb0, RB, M, nullptr, y, s);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_adjoint(pat_problem *p, int64_t R, const void *yhat, void *p_out, pat_precision prec, void *stream) {
    g_err.clear();
    if (!p || !yhat || !p_out || R < 1) return fail(PAT_ERR_INVALID_ARG, "pat_adjoint: NULL pointer or R < 1");
    pat::Prec pr;
    PAT_TRY(check_prec(prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int RB = fit_rb(p->ops.n, pr, choose_rb(R));
    PAT_TRY(check_block(p->ops.n, pr, RB));
    SweepWS *w;
    PAT_TRY(get_sweep(p, pr, RB, true, &w));
    const bool f64 = pr == pat::Prec::F64;
    if (!w->g_adj_user)
        PAT_TRY(capture(p, &w->g_adj_user, [&](hipStream_t cs) { enqueue_adjoint(p, *w, w->Y, f64, cs); }));
    const int64_t M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        pat::launch_pack(f64, f64, yhat, R, rb0, RB, M, nullptr, w->Y, s);
        PAT_HIP(hipGraphLaunch(w->g_adj_user, s));
        pat::launch_unpack(f64, f64, w->S[0], R, rb0, RB, p->ops.n, perm, p_out, s);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status rto_sample(pat_problem *p, const double *y_obs, const pat_rto_params *prm, int64_t S, double *samples,
                      double *mean, double *std, double *resid_hist, void *stream) {
    g_err.clear();
    if (!p || !y_obs || !prm || !samples || S < 1) return fail(PAT_ERR_INVALID_ARG, "rto_sample: NULL pointer or S < 1");
    PAT_TRY(check_rto_params(prm, S, std != nullptr));
    pat::Prec pr;
    PAT_TRY(check_prec(prm->sweep_prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);

    const int RB = prm->rhs_block ? prm->rhs_block : auto_rb(p->tuned, p->ops.n, S, pr);
    PAT_TRY(check_block(p->ops.n, pr, RB));
    PAT_TRY(check_spectral(p, prm, RB));
    const int n_iter = prm->n_iter;
    const bool lsqr = prm->solver == PAT_LSQR;
    const int64_t N = p->ops.n;

    Solve proto;
    PAT_TRY(make_solve(p, prm, pr, RB, S, 0, resid_hist, s, &proto));
    SweepWS *w = proto.w;
    PAT_TRY(solver_graphs(p, w, proto.c, proto.isig));
    std::vector<double> chk_host(size_t(((S + RB - 1) / RB) * RB), 0.0);
    size_t ev_used = 0;
    std::vector<int> ev_kind;  // per event pair: 0 forward, 1 transpose
    auto fwd = [&]() -> pat_status {
        PAT_TRY(launch_sweep(p, w->g_fwd_cgls, s, &ev_used));
        if (p->prof) ev_kind.push_back(0);
        return PAT_OK;
    };
    auto adj = [&]() -> pat_status {
        PAT_TRY(launch_sweep(p, w->g_adj_cgls, s, &ev_used));
        if (p->prof) ev_kind.push_back(1);
        return PAT_OK;
    };
    for (int64_t rb0 = 0; rb0 < S; rb0 += RB) {
        std::vector<Solve> blk{proto};
        blk[0].rb0 = rb0;
        build_rhs(blk[0], y_obs, prm);
        PAT_TRY(drive(blk, n_iter, fwd, adj));
        finish_block(blk[0], prm, samples);
        PAT_HIP(hipMemcpyAsync(chk_host.data() + rb0, ph_check(blk[0]), RB * sizeof(double), hipMemcpyDeviceToHost, s));
        PAT_TRY(final_check(blk[0], y_obs, prm, prm->final_resid));
    }
    if (mean || std) pat::launch_stats(samples, S, N, mean, std, s);
    PAT_HIP(hipGetLastError());
    PAT_HIP(hipStreamSynchronize(s));
    PAT_TRY(fold_profile(p, ev_kind));
    for (int64_t k = 0; k < S; ++k)
        if (!std::isfinite(chk_host[size_t(k)]))
            return fail(PAT_ERR_NONFINITE, std::string("non-finite ") + (lsqr ? "LSQR" : "CGLS") +
                                               " scalar for sample " + std::to_string(k));
    return PAT_OK;
}

pat_status pat_autotune(pat_problem *p, int64_t S, pat_precision prec, int32_t *rhs_block, double *step_us,
                        void *stream) {
    g_err.clear();
    if (!p || S < 1) return fail(PAT_ERR_INVALID_ARG, "pat_autotune: NULL handle or S < 1");
    pat::Prec pr;
    PAT_TRY(check_prec(prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    int rb = 0;
    double us = 0.0;
    TuneScope scope({p}, pr);
    const pat_status st = tune_rb({p}, p->cap, S, pr, static_cast<hipStream_t>(stream), &rb, &us);
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    scope.release_except(st == PAT_OK ? rb : -1);
    PAT_TRY(st);
    p->tuned[{S, int(pr)}] = rb;
    if (rhs_block) *rhs_block = rb;
    if (step_us) *step_us = us;
    return PAT_OK;
}

pat_status pat_batch_create(pat_problem *const *problems, int32_t n, pat_batch **out) {
    g_err.clear();
    if (!problems || !out || n < 1) return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: NULL pointer or n < 1");
    if (n > pat::kMaxMeshes)
        return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: at most " + std::to_string(pat::kMaxMeshes) + " problems");
    *out = nullptr;
    for (int32_t m = 0; m < n; ++m) {
        if (!problems[m]) return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: NULL problem");
        if (problems[m]->device != problems[0]->device)
            return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: problems on different devices");
        if (problems[m]->ops.n_steps != problems[0]->ops.n_steps)
            return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: problems need the same number of time steps");
        for (int32_t q = 0; q < m; ++q)
            if (problems[q] == problems[m]) return fail(PAT_ERR_INVALID_ARG, "pat_batch_create: repeated problem");
    }
    DeviceGuard guard(problems[0]->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    std::unique_ptr<pat_batch> b(new pat_batch());
    b->device = problems[0]->device;
    b->probs.assign(problems, problems + n);
    PAT_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    *out = b.release();
    return PAT_OK;
}

pat_status pat_batch_destroy(pat_batch *b) {
    if (!b) return PAT_OK;
    DeviceGuard guard(b->device);
    if (b->g_fwd) (void)hipGraphExecDestroy(b->g_fwd);
    if (b->g_adj) (void)hipGraphExecDestroy(b->g_adj);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return PAT_OK;
}

pat_status pat_batch_merge(pat_batch *b, int32_t forward, int32_t transpose) {
    g_err.clear();
    if (!b) return fail(PAT_ERR_INVALID_ARG, "pat_batch_merge: NULL handle");
    if (forward < -1 || forward > 2 || transpose < -1 || transpose > 2)
        return fail(PAT_ERR_INVALID_ARG, "pat_batch_merge: values must be -1, 0, 1 or 2");
    b->force_mf = forward;
    b->force_ma = transpose;
    return PAT_OK;
}

pat_status pat_batch_autotune(pat_batch *b, int64_t S, pat_precision prec, int32_t *rhs_block, double *step_us,
                              void *stream) {
    g_err.clear();
    if (!b || S < 1) return fail(PAT_ERR_INVALID_ARG, "pat_batch_autotune: NULL handle or S < 1");
    pat::Prec pr;
    PAT_TRY(check_prec(prec, &pr));
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    int rb = 0;
    double us = 0.0;
    int mf = 1, ma = 1;
    TuneScope scope(b->probs, pr);
    const pat_status st = tune_rb(b->probs, b->cap, S, pr, static_cast<hipStream_t>(stream), &rb, &us, &mf, &ma);
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    scope.release_except(st == PAT_OK ? rb : -1);
    PAT_TRY(st);
    b->tune[{S, int(pr)}] = pat_batch::Tune{rb, mf, ma};
    if (rhs_block) *rhs_block = rb;
    if (step_us) *step_us = us;
    return PAT_OK;
}

pat_status rto_sample_batch(pat_batch *b, const double *const *y_obs, const pat_rto_params *prm, const int64_t *S,
                            double *const *samples, double *const *mean, double *const *std,
                            double *const *resid_hist, void *stream) {
    g_err.clear();
    if (!b || !y_obs || !prm || !S || !samples) return fail(PAT_ERR_INVALID_ARG, "rto_sample_batch: NULL pointer");
    const size_t n = b->probs.size();
    int64_t smax = 0;
    for (size_t m = 0; m < n; ++m) {
        if (!y_obs[m] || !samples[m] || S[m] < 1)
            return fail(PAT_ERR_INVALID_ARG, "rto_sample_batch: NULL y_obs or samples, or S < 1, for problem " +
                                                 std::to_string(m));
        PAT_TRY(check_rto_params(&prm[m], S[m], std && std[m]));
        if (prm[m].n_iter != prm[0].n_iter || prm[m].reorth != prm[0].reorth ||
            prm[m].sweep_prec != prm[0].sweep_prec || prm[m].rhs_block != prm[0].rhs_block ||
            prm[m].solver != prm[0].solver)
            return fail(PAT_ERR_INVALID_ARG,
                        "rto_sample_batch: n_iter, reorth, sweep_prec, rhs_block and solver must agree");
        smax = std::max(smax, S[m]);
    }
    pat::Prec pr;
    PAT_TRY(check_prec(prm[0].sweep_prec, &pr));
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t nmax = 0;
    for (size_t m = 0; m < n; ++m) nmax = std::max<int64_t>(nmax, b->probs[m]->ops.n);
    int RB = prm[0].rhs_block ? prm[0].rhs_block : fit_rb(nmax, pr, choose_rb(smax));
    int mf = 1, ma = 1;
    {
        auto it = b->tune.find({smax, int(pr)});
        if (it != b->tune.end() && (prm[0].rhs_block == 0 || prm[0].rhs_block == it->second.rb)) {
            RB = it->second.rb;
            mf = it->second.mf;
            ma = it->second.ma;
        }
        if (b->force_mf >= 0) mf = b->force_mf;
        if (b->force_ma >= 0) ma = b->force_ma;
    }
    PAT_TRY(check_block(nmax, pr, RB));
    const int n_iter = prm[0].n_iter;
    const bool lsqr = prm[0].solver == PAT_LSQR;

    std::vector<Solve> proto(n);
    std::vector<SweepWS *> W(n);
    std::vector<CglsWS *> C(n);
    std::vector<double> scale(n);
    std::vector<void *> yout(n);
    std::vector<const void *> yin(n), kf, ka;
    for (size_t m = 0; m < n; ++m) {
        pat_problem *p = b->probs[m];
        PAT_TRY(check_spectral(p, &prm[m], RB));
        PAT_TRY(make_solve(p, &prm[m], pr, RB, S[m], 0, resid_hist ? resid_hist[m] : nullptr, s, &proto[m]));
        W[m] = proto[m].w;
        C[m] = proto[m].c;
        scale[m] = 1.0 / prm[m].sigma;
        yout[m] = C[m]->qd;
        yin[m] = C[m]->rd;
        kf.push_back(W[m]);
        kf.push_back(C[m]->qd);
        ka.push_back(W[m]);
        ka.push_back(C[m]->rd);
    }
    if (mf == 2 || ma == 2)  // whole sweeps per problem use each problem's own solver graphs
        for (size_t m = 0; m < n; ++m) PAT_TRY(solver_graphs(b->probs[m], W[m], C[m], scale[m]));
    if (mf != 2 && (!b->g_fwd || kf != b->key_fwd || scale != b->key_scale || (mf == 1) != b->key_mf)) {
        PAT_TRY(capture_on(b->cap, &b->g_fwd,
                           [&](hipStream_t cs) { enqueue_forward_multi(b->probs, W, yout, true, scale, cs, mf == 1); }));
        b->key_fwd = kf;
        b->key_scale = scale;
        b->key_mf = mf == 1;
    }
    if (ma != 2 && (!b->g_adj || ka != b->key_adj || (ma == 1) != b->key_ma)) {
        PAT_TRY(capture_on(b->cap, &b->g_adj,
                           [&](hipStream_t cs) { enqueue_adjoint_multi(b->probs, W, yin, true, cs, ma == 1); }));
        b->key_adj = ka;
        b->key_ma = ma == 1;
    }
    auto fwd = [&]() -> pat_status {
        if (mf == 2) {
            for (size_t m = 0; m < n; ++m) PAT_HIP(hipGraphLaunch(W[m]->g_fwd_cgls, s));
        } else {
            PAT_HIP(hipGraphLaunch(b->g_fwd, s));
        }
        return PAT_OK;
    };
    auto adj = [&]() -> pat_status {
        if (ma == 2) {
            for (size_t m = 0; m < n; ++m) PAT_HIP(hipGraphLaunch(W[m]->g_adj_cgls, s));
        } else {
            PAT_HIP(hipGraphLaunch(b->g_adj, s));
        }
        return PAT_OK;
    };
    std::vector<std::vector<double>> chk(n, std::vector<double>(size_t(((smax + RB - 1) / RB) * RB), 0.0));
    for (int64_t rb0 = 0; rb0 < smax; rb0 += RB) {
        std::vector<Solve> blk = proto;
        for (size_t m = 0; m < n; ++m) {
            blk[m].rb0 = rb0;
            build_rhs(blk[m], y_obs[m], &prm[m]);
        }
        PAT_TRY(drive(blk, n_iter, fwd, adj));
        for (size_t m = 0; m < n; ++m) {
            if (rb0 < S[m]) finish_block(blk[m], &prm[m], samples[m]);
            PAT_HIP(hipMemcpyAsync(chk[m].data() + rb0, ph_check(blk[m]), RB * sizeof(double), hipMemcpyDeviceToHost, s));
            if (rb0 < S[m]) PAT_TRY(final_check(blk[m], y_obs[m], &prm[m], prm[m].final_resid));
        }
    }
    for (size_t m = 0; m < n; ++m) {
        double *mm = mean ? mean[m] : nullptr, *sd = std ? std[m] : nullptr;
        if (mm || sd) pat::launch_stats(samples[m], S[m], b->probs[m]->ops.n, mm, sd, s);
    }
    PAT_HIP(hipGetLastError());
    PAT_HIP(hipStreamSynchronize(s));
    for (size_t m = 0; m < n; ++m)
        for (int64_t k = 0; k < S[m]; ++k)
            if (!std::isfinite(chk[m][size_t(k)]))
                return fail(PAT_ERR_NONFINITE, std::string("non-finite ") + (lsqr ? "LSQR" : "CGLS") +
                                                   " scalar for problem " + std::to_string(m) + " sample " +
                                                   std::to_string(k));
    return PAT_OK;
}

pat_status pat_spectral_prior_set(pat_problem *p, const pat_spectral_desc *d) {
    g_err.clear();
    if (!p) return fail(PAT_ERR_INVALID_ARG, "pat_spectral_prior_set: NULL handle");
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    PAT_HIP(hipDeviceSynchronize());
    // drop the previous prior and its work buffers
    for (void *a : p->spec_allocs) dev_free(p, a);
    p->spec_allocs.clear();
    for (auto &kv : p->specws) {
        dev_free(p, kv.second.gr);
        dev_free(p, kv.second.gc);
        dev_free(p, kv.second.ym);
        dev_free(p, kv.second.lx);
    }
    p->specws.clear();
    for (auto it = p->cgls.begin(); it != p->cgls.end();) {  // latent-space solver workspaces
        if (it->first.second != p->ops.n) {
            CglsWS &c = it->second;
            double *bufs[] = {c.x, c.d, c.s, c.rp, c.qp, c.rd, c.qd, c.Q, c.part, c.mpart, c.coef, c.scal, c.cg, c.gram,
                              c.v, c.zp, c.zd, c.lrp, c.lrd};
            for (double *q : bufs) dev_free(p, q);
            it = p->cgls.erase(it);
        } else {
            ++it;
        }
    }
    p->spec = false;
    p->sops = pat::SpecOps{};
    if (!d) return PAT_OK;
    const int n = d->n;
    if (n < 8 || n > 128 || (n & (n - 1)))
        return fail(PAT_ERR_INVALID_ARG, "spectral prior: n must be a power of two in [8, 128]");
    if (!(d->side > 0.0) || !(d->ell > 0.0) || !(d->sigma > 0.0) || !(d->expo > 0.0) || !std::isfinite(d->side) ||
        !std::isfinite(d->ell) || !std::isfinite(d->sigma) || !std::isfinite(d->expo) || !std::isfinite(d->lo[0]) ||
        !std::isfinite(d->lo[1]) || !std::isfinite(d->lo[2]))
        return fail(PAT_ERR_INVALID_ARG, "spectral prior: side, ell, sigma and expo must be positive and finite");
    const int64_t G = int64_t(n) * n * n, N = p->ops.n;
    const double h = d->side / n;
    // square-root spectrum a(k) = c (ell^-2 + |k|^2)^(-expo/2), c giving pointwise variance sigma^2
    std::vector<double> amp(static_cast<size_t>(G));
    double sum = 0.0;
    for (int64_t g = 0; g < G; ++g) {
        const int64_t f[3] = {g % n, (g / n) % n, g / (int64_t(n) * n)};
        double k2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double fa = double(f[a] < n / 2 ? f[a] : f[a] - n);
            const double ka = 2.0 * M_PI * fa / d->side;
            k2 += ka * ka;
        }
        amp[size_t(g)] = std::pow(1.0 / (d->ell * d->ell) + k2, -0.5 * d->expo);
        sum += amp[size_t(g)] * amp[size_t(g)];
    }
    const double c = d->sigma * std::sqrt(double(G) / sum);
    for (double &v : amp) v *= c;
    // the z pass reads a(k) line by line on the half spectrum: store it as
    // [(ky * nh + kx) * n + kz] for kx < nh = n/2 + 1, so each line's n values are contiguous
    const int nh = n / 2 + 1;
    std::vector<double> ampz(size_t(n) * nh * n);
    for (int ky = 0; ky < n; ++ky)
        for (int kx = 0; kx < nh; ++kx)
            for (int kz = 0; kz < n; ++kz)
                ampz[(size_t(ky) * nh + kx) * n + kz] = amp[(size_t(kz) * n + ky) * n + kx];
    std::vector<double> tw(static_cast<size_t>(n));  // (re, im) pairs of exp(-2 pi i j / n), j < n/2
    for (int j = 0; j < n / 2; ++j) {
        tw[size_t(2 * j)] = std::cos(2.0 * M_PI * j / n);
        tw[size_t(2 * j + 1)] = -std::sin(2.0 * M_PI * j / n);
    }
    // trilinear interpolation rows (internal node order) and their transpose by grid point
    std::vector<int32_t> ig(static_cast<size_t>(N) * 8);
    std::vector<double> iw(static_cast<size_t>(N) * 8);
    for (int64_t q = 0; q < N; ++q) {
        int64_t i0[3];
        double fr[3];
        for (int a = 0; a < 3; ++a) {
            const double t = (p->xyz[size_t(q) * 3 + a] - d->lo[a]) / h;
            if (!(t >= 0.0) || !(t < double(n)))
                return fail(PAT_ERR_INVALID_ARG, "spectral prior: a mesh node lies outside the grid box");
            i0[a] = int64_t(std::floor(t));
            fr[a] = t - double(i0[a]);
        }
        int c8 = 0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx, ++c8) {
                    const double wgt = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) * (dz ? fr[2] : 1.0 - fr[2]);
                    const int64_t ix = (i0[0] + dx) % n, iy = (i0[1] + dy) % n, iz = (i0[2] + dz) % n;
                    ig[size_t(q * 8 + c8)] = int32_t((iz * n + iy) * n + ix);
                    iw[size_t(q * 8 + c8)] = wgt;
                }
    }
    std::vector<int32_t> tptr(static_cast<size_t>(G) + 1, 0), tq(static_cast<size_t>(N) * 8);
    std::vector<double> tw8(static_cast<size_t>(N) * 8);
    for (int64_t e = 0; e < N * 8; ++e) ++tptr[size_t(ig[size_t(e)]) + 1];
    for (int64_t g = 0; g < G; ++g) tptr[size_t(g) + 1] += tptr[size_t(g)];
    std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t e = 0; e < N * 8; ++e) {
        const int32_t g = ig[size_t(e)];
        tq[size_t(fill[size_t(g)])] = int32_t(e / 8);
        tw8[size_t(fill[size_t(g)]++)] = iw[size_t(e)];
    }
    pat::SpecOps so;
    so.n = n;
    so.logn = 0;
    while ((1 << so.logn) < n) ++so.logn;
    so.G = G;
    const size_t before = p->allocs.size();
    auto up = [&](const auto &vec, const auto **field) -> pat_status {
        pat_status st = upload(p, vec, field);
        return st;
    };
    pat_status st = PAT_OK;
    if (st == PAT_OK) st = up(ampz, &so.amp);
    if (st == PAT_OK) st = up(tw, &so.tw);
    if (st == PAT_OK) st = up(ig, &so.ig);
    if (st == PAT_OK) st = up(iw, &so.iw);
    if (st == PAT_OK) st = up(tptr, &so.tptr);
    if (st == PAT_OK) st = up(tq, &so.tq);
    if (st == PAT_OK) st = up(tw8, &so.tw8);
    for (size_t k = before; k < p->allocs.size(); ++k) p->spec_allocs.push_back(p->allocs[k]);
    if (st != PAT_OK) {
        for (void *a : p->spec_allocs) dev_free(p, a);
        p->spec_allocs.clear();
        return st;
    }
    p->sops = so;
    p->spec_desc = *d;
    p->spec = true;
    return PAT_OK;
}

pat_status pat_spectral_apply(pat_problem *p, int64_t R, int transpose, const double *x, double *y, void *stream) {
    g_err.clear();
    if (!p || !x || !y || R < 1) return fail(PAT_ERR_INVALID_ARG, "pat_spectral_apply: NULL pointer or R < 1");
    if (!p->spec) return fail(PAT_ERR_INVALID_ARG, "pat_spectral_apply: no spectral prior set");
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int RB = choose_rb(R);
    SpecWS *sw;
    PAT_TRY(get_spec(p, RB, &sw));
    const int64_t N = p->ops.n, G = p->sops.G;
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        if (!transpose) {
            pat::launch_pack(true, true, x, R, rb0, RB, G, nullptr, sw->lx, s);
            pat::launch_spectral(p->sops, RB, sw->lx, sw->gr, sw->gc, pat::Prec::F64, sw->ym, N, s);
            pat::launch_unpack(true, true, sw->ym, R, rb0, RB, N, perm, y, s);
        } else {
            pat::launch_pack(true, true, x, R, rb0, RB, N, perm, sw->ym, s);
            pat::launch_spectral_t(p->sops, RB, sw->ym, pat::Prec::F64, 1.0, nullptr, sw->gr, sw->gc, sw->lx, s);
            pat::launch_unpack(true, true, sw->lx, R, rb0, RB, G, nullptr, y, s);
        }
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_draw_normals(uint64_t seed, int32_t kind, int64_t k0, int64_t S, int64_t len, double *out,
                            void *stream) {
    g_err.clear();
    if (kind != 0 && kind != 1) return fail(PAT_ERR_INVALID_ARG, "pat_draw_normals: kind must be 0 or 1");
    if (S < 0 || len < 0 || k0 < 0) return fail(PAT_ERR_INVALID_ARG, "pat_draw_normals: negative size or offset");
    if (S == 0 || len == 0) return PAT_OK;
    if (!out) return fail(PAT_ERR_INVALID_ARG, "pat_draw_normals: NULL output");
    pat::launch_normals(seed, kind, k0, S, len, out, static_cast<hipStream_t>(stream));
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_solver_diagnostics(const double *diag, int64_t S, int32_t n_iter, int64_t n_data, double tau,
                                  double *data, double *prior, double *ext, int32_t *first, void *stream) {
    g_err.clear();
    if (!diag || S < 0 || n_iter < 0 || n_data < 1)
        return fail(PAT_ERR_INVALID_ARG, "pat_solver_diagnostics: NULL history, negative sizes or n_data < 1");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(PAT_ERR_INVALID_ARG, "pat_solver_diagnostics: tau must be >= 0");
    if (S == 0) return PAT_OK;
    pat::launch_diagnostics(diag, S, n_iter + 1, n_data, tau, data, prior, ext, first, static_cast<hipStream_t>(stream));
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_prior_apply(pat_problem *p, int64_t R, double prior_a, int transpose, const double *x, double *y,
                           void *stream) {
    g_err.clear();
    if (!p || !x || !y || R < 1) return fail(PAT_ERR_INVALID_ARG, "pat_prior_apply: NULL pointer or R < 1");
    if (x == y) return fail(PAT_ERR_INVALID_ARG, "pat_prior_apply: y must not alias x");
    if (!(prior_a >= 0.0) || !std::isfinite(prior_a)) return fail(PAT_ERR_INVALID_ARG, "prior_a must be >= 0");
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int RB = choose_rb(R);
    // the f64 sweep workspace of this block width holds the packed operands
    SweepWS *w;
    PAT_TRY(get_sweep(p, pat::Prec::F64, RB, false, &w));
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    const int64_t N = p->ops.n;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        pat::launch_pack(true, true, x, R, rb0, RB, N, perm, w->S[0], s);
        if (transpose)
            pat::launch_prior_t(p->ops, RB, prior_a, static_cast<const double *>(w->S[0]), static_cast<double *>(w->S[1]), s);
        else
            pat::launch_prior(p->ops, RB, prior_a, static_cast<const double *>(w->S[0]), static_cast<double *>(w->S[1]), s);
        pat::launch_unpack(true, true, w->S[1], R, rb0, RB, N, perm, y, s);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status pat_host_assemble(const pat_problem_desc *desc, int64_t *nnz_out, int32_t *rowptr, int32_t *col,
                             double *kval, double *k1val, double *bval, double *mass, int32_t *snode, double *sw,
                             double *lambda_max) {
    g_err.clear();
    if (!desc || !nnz_out) return fail(PAT_ERR_INVALID_ARG, "NULL descriptor or size output");
    pat::HostProblem hp;
    std::string err;
    pat_status st = pat::build_host_problem(*desc, hp, err);
    if (st != PAT_OK) return fail(st, err);
    const int32_t N = hp.n;
    *nnz_out = hp.rowptr.back();
    if (!rowptr) return PAT_OK;
    // rows in the caller's numbering: user row u = perm[i]; columns mapped the same way
    std::vector<int32_t> len(N);
    for (int32_t i = 0; i < N; ++i) len[hp.perm[i]] = hp.rowptr[i + 1] - hp.rowptr[i];
    rowptr[0] = 0;
    for (int32_t u = 0; u < N; ++u) rowptr[u + 1] = rowptr[u] + len[u];
    for (int32_t i = 0; i < N; ++i) {
        const int32_t u = hp.perm[i];
        std::vector<std::pair<int32_t, int32_t>> ent;
        for (int32_t k = hp.rowptr[i]; k < hp.rowptr[i + 1]; ++k) ent.push_back({hp.perm[hp.col[k]], k});
        std::sort(ent.begin(), ent.end());
        for (size_t q = 0; q < ent.size(); ++q) {
            const int32_t k = ent[q].second, o = rowptr[u] + int32_t(q);
            col[o] = ent[q].first;
            if (kval) kval[o] = hp.kval[k];
            if (k1val) k1val[o] = hp.k1val[k];
            if (bval) bval[o] = hp.boff[i] >= 0 ? hp.bval[hp.boff[i] + (k - hp.rowptr[i])] : 0.0;
        }
        if (mass) mass[u] = hp.mass[i];
    }
    for (int32_t s = 0; s < hp.n_obs; ++s)
        for (int k = 0; k < 4; ++k) {
            if (snode) snode[4 * s + k] = hp.perm[hp.snode[4 * s + k]];
            if (sw) sw[4 * s + k] = hp.sw[4 * s + k];
        }
    if (lambda_max) *lambda_max = hp.lambda_max;
    return PAT_OK;
}

pat_status pat_profile_enable(pat_problem *p, int enable) {
    if (!p) return fail(PAT_ERR_INVALID_ARG, "NULL handle");
    p->prof = enable != 0;
    p->prof_acc = pat_profile{};
    return PAT_OK;
}

pat_status pat_profile_get(const pat_problem *p, pat_profile *out) {
    if (!p || !out) return fail(PAT_ERR_INVALID_ARG, "NULL handle or output");
    *out = p->prof_acc;
    return PAT_OK;
}

pat_status pat_sync(pat_problem *p) {
    if (!p) return fail(PAT_ERR_INVALID_ARG, "NULL handle");
    DeviceGuard guard(p->device);
    PAT_HIP(hipDeviceSynchronize());
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

}  // extern "C"
