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
#include <map>
#include <memory>
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

bool valid_rb(int rb) { return rb == 1 || rb == 2 || rb == 4 || rb == 8 || rb == 16 || rb == 32 || rb == 64; }

size_t tsize(pat::Prec p) { return p == pat::Prec::F64 ? 8 : 4; }

}  // namespace

struct SweepWS {
    pat::Prec prec = pat::Prec::F64;
    int RB = 0;
    void *P[2] = {nullptr, nullptr};
    void *V[2] = {nullptr, nullptr};
    void *Y = nullptr;  // [M][RB] staging of the user-facing calls
    hipGraphExec_t g_fwd_user = nullptr, g_adj_user = nullptr;
    hipGraphExec_t g_fwd_cgls = nullptr, g_adj_cgls = nullptr;
    double g_fwd_cgls_scale = 0.0;
    const void *g_fwd_cgls_out = nullptr, *g_adj_cgls_in = nullptr;
};

struct CglsWS {
    int RB = 0;
    int cap_iter = -1;
    double *x = nullptr, *d = nullptr, *s = nullptr, *rp = nullptr, *qp = nullptr;
    double *rd = nullptr, *qd = nullptr, *Q = nullptr;
    double *part = nullptr, *mpart = nullptr, *coef = nullptr, *scal = nullptr;
    // LSQR: right vector v; z = G_ext w and the residual r = b - G_ext x, kept only for the histories
    double *v = nullptr, *zp = nullptr, *zd = nullptr, *lrp = nullptr, *lrd = nullptr;
};

struct pat_problem {
    int device = 0;
    pat::DevOps ops;
    pat_problem_info info{};
    bool perm_identity = true;
    std::vector<void *> allocs;
    std::map<std::pair<int, int>, SweepWS> sweeps;
    std::map<int, CglsWS> cgls;
    hipStream_t cap = nullptr;
    int64_t bytes = 0;
    // sweep timing
    bool prof = false;
    pat_profile prof_acc{};
    std::vector<hipEvent_t> events;
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
    p->bytes += int64_t(bytes);
    return PAT_OK;
}

void dev_free(pat_problem *p, void *ptr) {
    if (!ptr) return;
    for (auto &a : p->allocs)
        if (a == ptr) a = nullptr;
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
        w.prec = prec;
        w.RB = RB;
        const size_t bytes = size_t(p->ops.n) * RB * tsize(prec);
        for (int k = 0; k < 2; ++k) {
            PAT_TRY(dev_alloc(p, &w.P[k], bytes));
            PAT_TRY(dev_alloc(p, &w.V[k], bytes));
        }
    }
    if (need_y && !w.Y) {
        PAT_TRY(dev_alloc(p, &w.Y, size_t(p->ops.n_steps) * p->ops.n_obs * RB * tsize(prec)));
    }
    *out = &w;
    return PAT_OK;
}

// Capture the N_T launches of one sweep on the handle's capture stream.
template <class F>
pat_status capture(pat_problem *p, hipGraphExec_t *exec, F &&body) {
    if (*exec) {
        (void)hipGraphExecDestroy(*exec);
        *exec = nullptr;
    }
    PAT_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    body(p->cap);
    hipGraph_t g = nullptr;
    PAT_HIP(hipStreamEndCapture(p->cap, &g));
    hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PAT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return PAT_OK;
}

// Forward sweep: input state in w.P[0]; y^n (n = 1..N_T) written to y_out [N_T][N_obs][RB].
void enqueue_forward(pat_problem *p, SweepWS &w, void *y_out, bool y_f64, double yscale, hipStream_t s) {
    const pat::DevOps &op = p->ops;
    pat::launch_fwd_step(w.prec, w.RB, op, w.P[0], w.V[0], w.P[1], w.V[1], true, true, false, 0, y_out, y_f64,
                         yscale, s);
    int cur = 1;
    for (int n = 2; n <= op.n_steps; ++n) {
        pat::launch_fwd_step(w.prec, w.RB, op, w.P[cur], w.V[cur], w.P[1 - cur], w.V[1 - cur], true, false, true,
                             n - 2, y_out, y_f64, yscale, s);
        cur = 1 - cur;
    }
    pat::launch_fwd_step(w.prec, w.RB, op, w.P[cur], w.V[cur], nullptr, nullptr, false, false, true, op.n_steps - 1,
                         y_out, y_f64, yscale, s);
}

// Transpose sweep: data yhat [N_T][N_obs][RB]; result G^T yhat in w.P[0].
void enqueue_adjoint(pat_problem *p, SweepWS &w, const void *yhat, bool y_f64, hipStream_t s) {
    const pat::DevOps &op = p->ops;
    pat::launch_adj_init(w.prec, w.RB, op, w.P[0], w.V[0], yhat, y_f64, 1.0, s);
    int cur = 0;
    for (int n = op.n_steps; n >= 2; --n) {
        pat::launch_adj_step(w.prec, w.RB, op, w.P[0], w.V[cur], w.V[1 - cur], false, n - 2, yhat, y_f64, 1.0, s);
        cur = 1 - cur;
    }
    pat::launch_adj_step(w.prec, w.RB, op, w.P[0], w.V[cur], nullptr, true, 0, yhat, y_f64, 1.0, s);
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

pat_status get_cgls(pat_problem *p, int RB, int n_iter, bool reorth, bool lsqr, bool track, CglsWS **out) {
    CglsWS &c = p->cgls[RB];
    const int64_t N = p->ops.n, M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    if (c.RB == 0) {
        c.RB = RB;
        void *v;
        double **vec[] = {&c.x, &c.d, &c.s, &c.rp, &c.qp};
        for (double **q : vec) {
            PAT_TRY(dev_alloc(p, &v, size_t(N) * RB * 8));
            *q = static_cast<double *>(v);
        }
        PAT_TRY(dev_alloc(p, &v, size_t(M) * RB * 8)); c.rd = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(M) * RB * 8)); c.qd = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(4) * pat::kDotBlocks * RB * 8)); c.part = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(16) * RB * 8)); c.scal = static_cast<double *>(v);
    }
    if (lsqr && !c.v) {
        void *v;
        PAT_TRY(dev_alloc(p, &v, size_t(N) * RB * 8)); c.v = static_cast<double *>(v);
    }
    if (lsqr && track && !c.zd) {
        void *v;
        PAT_TRY(dev_alloc(p, &v, size_t(N) * RB * 8)); c.zp = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(N) * RB * 8)); c.lrp = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(M) * RB * 8)); c.zd = static_cast<double *>(v);
        PAT_TRY(dev_alloc(p, &v, size_t(M) * RB * 8)); c.lrd = static_cast<double *>(v);
    }
    const int need = reorth ? n_iter + 1 : 0;
    if (need > c.cap_iter) {
        dev_free(p, c.Q); dev_free(p, c.mpart); dev_free(p, c.coef);
        c.Q = c.mpart = c.coef = nullptr;
        void *v;
        if (need > 0) {
            PAT_TRY(dev_alloc(p, &v, size_t(need) * N * RB * 8)); c.Q = static_cast<double *>(v);
            PAT_TRY(dev_alloc(p, &v, size_t(need) * pat::kDotBlocks * RB * 8)); c.mpart = static_cast<double *>(v);
            PAT_TRY(dev_alloc(p, &v, size_t(need) * RB * 8)); c.coef = static_cast<double *>(v);
        }
        c.cap_iter = need;
    }
    *out = &c;
    return PAT_OK;
}


// State shared by the per-block solvers of rto_sample.
struct Solve {
    pat_problem *p;
    SweepWS *w;
    CglsWS *c;
    pat::Prec pr;
    int RB, n_iter;
    bool reorth;
    double isig, a;
    int64_t N, M, ld, S;
    double *resid_hist, *diag_hist;
    hipStream_t s;
    size_t *ev_used;
    std::vector<int> *ev_kind;
};

pat_status sweep(Solve &v, bool forward) {
    PAT_TRY(launch_sweep(v.p, forward ? v.w->g_fwd_cgls : v.w->g_adj_cgls, v.s, v.ev_used));
    if (v.p->prof) v.ev_kind->push_back(forward ? 0 : 1);
    return PAT_OK;
}

// Residual history column `it` from the data part rd [M][RB] and prior part rp [N][RB].
void record(Solve &v, const double *rd, const double *rp, int it, int64_t rb0) {
    if (!v.resid_hist && !v.diag_hist) return;
    double *pA = v.c->part, *pB = v.c->part + pat::kDotBlocks * v.RB;
    double *t1 = v.c->scal + 14 * v.RB, *t2 = v.c->scal + 15 * v.RB;
    pat::launch_dot_partial(rd, rd, v.M, v.RB, pA, v.s);
    pat::launch_dot_partial(rp, rp, v.N, v.RB, pB, v.s);
    pat::launch_dot_final(pA, nullptr, v.RB, t1, v.s);
    pat::launch_dot_final(pB, nullptr, v.RB, t2, v.s);
    pat::launch_resid(t1, t2, v.resid_hist, v.diag_hist, v.ld, it, rb0, v.S, v.RB, v.s);
}

// s = G_ext^T (rd, up) = G^T rd / sigma + L^T up; the transpose graph reads rd.
pat_status apply_gext_t(Solve &v, const double *up) {
    PAT_TRY(sweep(v, false));
    pat::launch_gext_t_combine(v.pr, v.p->ops, v.RB, v.a, v.isig, v.w->P[0], up, v.c->s, v.s);
    return PAT_OK;
}

// s -= sum_j (Q_j . s) Q_j over j < k, classical Gram-Schmidt applied twice.
void reorthogonalise(Solve &v, int k) {
    if (!v.reorth || k <= 0) return;
    for (int pass = 0; pass < 2; ++pass) {
        pat::launch_multidot(v.c->Q, v.c->s, k, v.N, v.RB, v.c->mpart, v.c->coef, v.s);
        pat::launch_project(v.c->Q, v.c->s, v.c->coef, k, v.N, v.RB, v.s);
    }
}

// qd = G x / sigma (through the forward graph), qp = L x.
pat_status apply_gext(Solve &v, const double *x) {
    pat::launch_cast_to_state(v.pr, x, v.w->P[0], v.N * v.RB, v.s);
    PAT_TRY(sweep(v, true));
    pat::launch_prior(v.p->ops, v.RB, v.a, x, v.c->qp, v.s);
    return PAT_OK;
}

// CGLS on one block; b in (rd, rp), x = 0 on entry.  Normal-equation residuals
// s_j are kept orthogonal by two classical Gram-Schmidt passes (App. A).
pat_status cgls_block(Solve &v, int64_t rb0, const double **chk) {
    CglsWS *c = v.c;
    const int RB = v.RB;
    double *gamma = c->scal, *delta = c->scal + RB, *alpha = c->scal + 2 * RB, *beta = c->scal + 3 * RB;
    double *invn = c->scal + 4 * RB, *gnew = c->scal + 5 * RB;
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * RB;
    record(v, c->rd, c->rp, 0, rb0);
    // s_0 = G_ext^T r_0
    PAT_TRY(apply_gext_t(v, c->rp));
    pat::launch_dot_partial(c->s, c->s, v.N, RB, pA, v.s);
    pat::launch_dot_final(pA, nullptr, RB, gnew, v.s);
    pat::launch_scalar_gamma(gamma, gnew, beta, invn, 1, RB, v.s);
    pat::launch_append_dir(c->s, v.reorth ? c->Q : nullptr, c->d, invn, beta, 1, v.N, RB, v.s);
    for (int it = 1; it <= v.n_iter; ++it) {
        // q = G_ext d ; alpha = gamma / ||q||^2 ; x += alpha d ; r -= alpha q
        PAT_TRY(apply_gext(v, c->d));
        pat::launch_dot_partial(c->qd, c->qd, v.M, RB, pA, v.s);
        pat::launch_dot_partial(c->qp, c->qp, v.N, RB, pB, v.s);
        pat::launch_dot_final(pA, pB, RB, delta, v.s);
        pat::launch_scalar_alpha(gamma, delta, alpha, RB, v.s);
        pat::launch_update_xr(c->x, c->d, c->rp, c->qp, alpha, v.N, RB, v.s);
        pat::launch_axpy_neg(c->rd, c->qd, alpha, v.M, RB, v.s);
        record(v, c->rd, c->rp, it, rb0);
        if (it == v.n_iter) break;
        // s = G_ext^T r ; beta = gamma_new / gamma ; d = s + beta d
        PAT_TRY(apply_gext_t(v, c->rp));
        reorthogonalise(v, it);
        pat::launch_dot_partial(c->s, c->s, v.N, RB, pA, v.s);
        pat::launch_dot_final(pA, nullptr, RB, gnew, v.s);
        pat::launch_scalar_gamma(gamma, gnew, beta, invn, 0, RB, v.s);
        pat::launch_append_dir(c->s, v.reorth ? c->Q + size_t(it) * v.N * RB : nullptr, c->d, invn, beta, 0, v.N, RB,
                               v.s);
    }
    *chk = gamma;
    return PAT_OK;
}

// LSQR on one block (Paige and Saunders' bidiagonalisation, the solver of
// Sec. 5.2).  b in (rd, rp), x = 0 on entry.  The left vector u lives in
// (rd, rp), so the transpose graph reads it where CGLS keeps its residual; the
// search direction w lives in d.  The residual r = b - G_ext x is carried
// (through z = G_ext w) only when a history is asked for.
pat_status lsqr_block(Solve &v, int64_t rb0, const double **chk) {
    CglsWS *c = v.c;
    const int RB = v.RB;
    const int64_t N = v.N, M = v.M;
    const bool track = v.resid_hist || v.diag_hist;
    double *sc = c->scal;
    pat::LsqrScalars L{sc, sc + RB, sc + 2 * RB, sc + 3 * RB, sc + 4 * RB, sc + 5 * RB,
                       sc + 6 * RB, sc + 7 * RB, sc + 8 * RB, sc + 9 * RB, sc + 10 * RB, sc + 11 * RB};
    double *n1 = sc + 12 * RB, *n2 = sc + 13 * RB;
    double *pA = c->part, *pB = c->part + pat::kDotBlocks * RB;
    if (track) {
        pat::launch_lincomb(c->lrd, c->rd, nullptr, 1.0, nullptr, nullptr, 0.0, M, RB, v.s);
        pat::launch_lincomb(c->lrp, c->rp, nullptr, 1.0, nullptr, nullptr, 0.0, N, RB, v.s);
        record(v, c->lrd, c->lrp, 0, rb0);
    }
    // beta_1 u_1 = b
    pat::launch_dot_partial(c->rd, c->rd, M, RB, pA, v.s);
    pat::launch_dot_partial(c->rp, c->rp, N, RB, pB, v.s);
    pat::launch_dot_final(pA, nullptr, RB, n1, v.s);
    pat::launch_dot_final(pB, nullptr, RB, n2, v.s);
    pat::launch_lsqr_scalar(pat::LsqrStage::InitBeta, L, n1, n2, RB, v.s);
    pat::launch_lincomb(c->rd, c->rd, L.inv, 1.0, nullptr, nullptr, 0.0, M, RB, v.s);
    pat::launch_lincomb(c->rp, c->rp, L.inv, 1.0, nullptr, nullptr, 0.0, N, RB, v.s);
    // alpha_1 v_1 = G_ext^T u_1 ; w_1 = v_1
    PAT_TRY(apply_gext_t(v, c->rp));
    pat::launch_dot_partial(c->s, c->s, N, RB, pA, v.s);
    pat::launch_dot_final(pA, nullptr, RB, n1, v.s);
    pat::launch_lsqr_scalar(pat::LsqrStage::InitAlpha, L, n1, nullptr, RB, v.s);
    pat::launch_lsqr_vw(c->s, L.inv, L.zfac, c->v, c->d, v.reorth ? c->Q : nullptr, 1, N, RB, v.s);
    for (int k = 1; k <= v.n_iter; ++k) {
        // q = G_ext v_k ; z_k = q - zfac z_{k-1}
        PAT_TRY(apply_gext(v, c->v));
        if (track) {
            pat::launch_lincomb(c->zd, c->qd, nullptr, 1.0, k > 1 ? c->zd : nullptr, L.zfac, -1.0, M, RB, v.s);
            pat::launch_lincomb(c->zp, c->qp, nullptr, 1.0, k > 1 ? c->zp : nullptr, L.zfac, -1.0, N, RB, v.s);
        }
        // beta_{k+1} u_{k+1} = q - alpha_k u_k ; rotation
        pat::launch_lincomb(c->rd, c->qd, nullptr, 1.0, c->rd, L.alpha, -1.0, M, RB, v.s);
        pat::launch_lincomb(c->rp, c->qp, nullptr, 1.0, c->rp, L.alpha, -1.0, N, RB, v.s);
        pat::launch_dot_partial(c->rd, c->rd, M, RB, pA, v.s);
        pat::launch_dot_partial(c->rp, c->rp, N, RB, pB, v.s);
        pat::launch_dot_final(pA, nullptr, RB, n1, v.s);
        pat::launch_dot_final(pB, nullptr, RB, n2, v.s);
        pat::launch_lsqr_scalar(pat::LsqrStage::Beta, L, n1, n2, RB, v.s);
        pat::launch_lincomb(c->rd, c->rd, L.inv, 1.0, nullptr, nullptr, 0.0, M, RB, v.s);
        pat::launch_lincomb(c->rp, c->rp, L.inv, 1.0, nullptr, nullptr, 0.0, N, RB, v.s);
        // x += (phi/rho) w ; r -= (phi/rho) z
        pat::launch_lincomb(c->x, c->x, nullptr, 1.0, c->d, L.step, 1.0, N, RB, v.s);
        if (track) {
            pat::launch_lincomb(c->lrd, c->lrd, nullptr, 1.0, c->zd, L.step, -1.0, M, RB, v.s);
            pat::launch_lincomb(c->lrp, c->lrp, nullptr, 1.0, c->zp, L.step, -1.0, N, RB, v.s);
            record(v, c->lrd, c->lrp, k, rb0);
        }
        if (k == v.n_iter) break;
        // alpha_{k+1} v_{k+1} = G_ext^T u_{k+1} - beta_{k+1} v_k, reorthogonalised
        PAT_TRY(apply_gext_t(v, c->rp));
        pat::launch_lincomb(c->s, c->s, nullptr, 1.0, c->v, L.beta, -1.0, N, RB, v.s);
        reorthogonalise(v, k);
        pat::launch_dot_partial(c->s, c->s, N, RB, pA, v.s);
        pat::launch_dot_final(pA, nullptr, RB, n1, v.s);
        pat::launch_lsqr_scalar(pat::LsqrStage::Alpha, L, n1, nullptr, RB, v.s);
        pat::launch_lsqr_vw(c->s, L.inv, L.zfac, c->v, c->d, v.reorth ? c->Q + size_t(k) * N * RB : nullptr, 0, N, RB,
                            v.s);
    }
    *chk = L.phib;
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
    UP(hp.ell_val, ell_val64);
    UP(hp.xval, xval64);
    UP(hp.bslot, bslot64);
    UP(to_f32(hp.ell_val), ell_val32);
    UP(to_f32(hp.xval), xval32);
    UP(to_f32(hp.bslot), bslot32);
#undef UP
    p->perm_identity = true;
    for (int32_t i = 0; i < hp.n; ++i)
        if (hp.perm[i] != i) p->perm_identity = false;
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
        hipGraphExec_t *gs[] = {&w.g_fwd_user, &w.g_adj_user, &w.g_fwd_cgls, &w.g_adj_cgls};
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
    const int RB = choose_rb(R);
    SweepWS *w;
    PAT_TRY(get_sweep(p, pr, RB, true, &w));
    if (!w->g_fwd_user)
        PAT_TRY(capture(p, &w->g_fwd_user, [&](hipStream_t cs) { enqueue_forward(p, *w, w->Y, false, 1.0, cs); }));
    const bool f64 = pr == pat::Prec::F64;
    const int64_t M = int64_t(p->ops.n_steps) * p->ops.n_obs;
    const int32_t *perm = p->perm_identity ? nullptr : p->ops.perm;
    for (int64_t rb0 = 0; rb0 < R; rb0 += RB) {
        pat::launch_pack(f64, f64, p0, R, rb0, RB, p->ops.n, perm, w->P[0], s);
        PAT_HIP(hipGraphLaunch(w->g_fwd_user, s));
        pat::launch_unpack(f64, f64, w->Y, R, rb0, RB, M, nullptr, y, s);
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
    const int RB = choose_rb(R);
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
        pat::launch_unpack(f64, f64, w->P[0], R, rb0, RB, p->ops.n, perm, p_out, s);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

pat_status rto_sample(pat_problem *p, const double *y_obs, const pat_rto_params *prm, int64_t S, double *samples,
                      double *mean, double *std, double *resid_hist, void *stream) {
    g_err.clear();
    if (!p || !y_obs || !prm || !samples || S < 1) return fail(PAT_ERR_INVALID_ARG, "rto_sample: NULL pointer or S < 1");
    if ((prm->eta == nullptr) != (prm->xi == nullptr))
        return fail(PAT_ERR_INVALID_ARG, "rto_sample: pass both eta and xi, or neither (device draws)");
    if (prm->sample0 < 0) return fail(PAT_ERR_INVALID_ARG, "rto_sample: sample0 must be >= 0");
    if (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma)) return fail(PAT_ERR_INVALID_ARG, "sigma must be > 0");
    if (!(prm->prior_a >= 0.0) || !std::isfinite(prm->prior_a)) return fail(PAT_ERR_INVALID_ARG, "prior_a must be >= 0");
    if (prm->n_iter < 1) return fail(PAT_ERR_INVALID_ARG, "n_iter must be >= 1");
    if (std && S < 2) return fail(PAT_ERR_INVALID_ARG, "std needs S >= 2");
    if (prm->rhs_block != 0 && !valid_rb(prm->rhs_block))
        return fail(PAT_ERR_INVALID_ARG, "rhs_block must be 0 or a power of two <= 64");
    if (prm->solver != PAT_CGLS && prm->solver != PAT_LSQR)
        return fail(PAT_ERR_INVALID_ARG, "solver must be PAT_CGLS or PAT_LSQR");
    pat::Prec pr;
    PAT_TRY(check_prec(prm->sweep_prec, &pr));
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(PAT_ERR_HIP, "cannot select the device");
    hipStream_t s = static_cast<hipStream_t>(stream);

    const int RB = prm->rhs_block ? prm->rhs_block : choose_rb(S);
    const int n_iter = prm->n_iter;
    const bool reorth = prm->reorth != 0;
    const pat::DevOps &op = p->ops;
    const int64_t N = op.n, M = int64_t(op.n_steps) * op.n_obs;
    const double isig = 1.0 / prm->sigma, a = prm->prior_a;
    const int32_t *perm = p->perm_identity ? nullptr : op.perm;

    SweepWS *w;
    PAT_TRY(get_sweep(p, pr, RB, false, &w));
    const bool lsqr = prm->solver == PAT_LSQR;
    CglsWS *c;
    PAT_TRY(get_cgls(p, RB, n_iter, reorth, lsqr, resid_hist || prm->diag_hist, &c));
    if (!w->g_fwd_cgls || w->g_fwd_cgls_scale != isig || w->g_fwd_cgls_out != c->qd) {
        PAT_TRY(capture(p, &w->g_fwd_cgls, [&](hipStream_t cs) { enqueue_forward(p, *w, c->qd, true, isig, cs); }));
        w->g_fwd_cgls_scale = isig;
        w->g_fwd_cgls_out = c->qd;
    }
    if (!w->g_adj_cgls || w->g_adj_cgls_in != c->rd) {
        PAT_TRY(capture(p, &w->g_adj_cgls, [&](hipStream_t cs) { enqueue_adjoint(p, *w, c->rd, true, cs); }));
        w->g_adj_cgls_in = c->rd;
    }
    const int64_t ld = n_iter + 1;
    std::vector<double> chk_host(size_t(((S + RB - 1) / RB) * RB), 0.0);
    // event pairs: even index = forward sweep, odd = transpose sweep, per kind in order
    size_t ev_used = 0;
    std::vector<int> ev_kind;  // 0 forward, 1 transpose, per event pair
    Solve sv{p, w, c, pr, RB, n_iter, reorth, isig, a, N, M, ld, S, resid_hist, prm->diag_hist, s, &ev_used, &ev_kind};

    for (int64_t rb0 = 0; rb0 < S; rb0 += RB) {
        // right-hand side b = (y_obs/sigma + eta, xi) in (rd, rp)
        if (prm->eta) {
            pat::launch_build_rhs(y_obs, prm->eta, S, rb0, RB, M, isig, c->rd, s);
            pat::launch_pack(true, true, prm->xi, S, rb0, RB, N, perm, c->rp, s);
        } else {
            pat::launch_build_rhs_rng(y_obs, prm->seed, prm->sample0, S, rb0, RB, M, isig, c->rd, s);
            pat::launch_xi_rng(prm->seed, prm->sample0, S, rb0, RB, N, perm, c->rp, s);
        }
        pat::launch_fill(c->x, N * RB, 0.0, s);
        const double *chk = nullptr;
        if (lsqr) {
            PAT_TRY(lsqr_block(sv, rb0, &chk));
        } else {
            PAT_TRY(cgls_block(sv, rb0, &chk));
        }
        pat::launch_unpack(true, true, c->x, S, rb0, RB, N, perm, samples, s);
        PAT_HIP(hipMemcpyAsync(chk_host.data() + rb0, chk, RB * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (mean || std) pat::launch_stats(samples, S, N, mean, std, s);
    PAT_HIP(hipGetLastError());
    PAT_HIP(hipStreamSynchronize(s));
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
    for (int64_t k = 0; k < S; ++k)
        if (!std::isfinite(chk_host[size_t(k)]))
            return fail(PAT_ERR_NONFINITE, std::string("non-finite ") + (lsqr ? "LSQR" : "CGLS") +
                                               " scalar for sample " + std::to_string(k));
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
        pat::launch_pack(true, true, x, R, rb0, RB, N, perm, w->P[0], s);
        if (transpose)
            pat::launch_prior_t(p->ops, RB, prior_a, static_cast<const double *>(w->P[0]), static_cast<double *>(w->P[1]), s);
        else
            pat::launch_prior(p->ops, RB, prior_a, static_cast<const double *>(w->P[0]), static_cast<double *>(w->P[1]), s);
        pat::launch_unpack(true, true, w->P[1], R, rb0, RB, N, perm, y, s);
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
