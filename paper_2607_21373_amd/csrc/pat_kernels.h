// Kernel launch interface of libpat (implemented in pat_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pat {

// Device copy of the assembled operators (internal node numbering).
struct DevOps {
    int32_t n = 0, n_obs = 0, n_steps = 0;
    int64_t nnz = 0;
    // CSR pattern of K with the unit-coefficient stiffness K1 (prior factor)
    const int32_t *rowptr = nullptr, *col = nullptr;
    const double *k1val64 = nullptr;
    const int32_t *snode = nullptr, *injptr = nullptr, *injs = nullptr, *perm = nullptr;
    const double *dtm64 = nullptr, *sqrtm = nullptr, *isqrtm = nullptr, *sw64 = nullptr, *injw64 = nullptr;
    const float *dtm32 = nullptr, *sw32 = nullptr, *injw32 = nullptr;
    // padded row layout of K for the time-step kernels
    const int32_t *ell_col = nullptr, *xptr = nullptr, *xcol = nullptr, *bsoff = nullptr, *bnum = nullptr;
    const double *ell_val64 = nullptr, *xval64 = nullptr, *bslot64 = nullptr;
    const float *ell_val32 = nullptr, *xval32 = nullptr, *bslot32 = nullptr;
    // halo tiles of the float32 step kernels (HaloTiles)
    const int32_t *ht_desc = nullptr, *ht_hrow = nullptr;
    const uint32_t *ht_meta = nullptr;
    int32_t n_ht = 0;
    int32_t n_cu = 0;  // compute units of the device (the halo kernels keep two workgroups on each)
    double dt = 0.0;
};

enum class Prec { F64, F32 };


// One forward Stormer-Verlet step in the three-level form (Sec. 3 eq. (fully-discrete),
// lumped mass, S^n = p^{n+1/2}):
//   Sn = S + (S - Sp) - (dt/m)(dt K S + B (S - Sp)),
// optionally sampling y = Pi (S + Sp)/2 (= Pi p^n) of the incoming state into
// y_out[(t*n_obs + s)*RB + r] * yscale.  The first step of a sweep passes Sp == S
// (v^0 = 0).  rows = 0 launches only the sampling part.  S, Sp and Sn are three
// distinct buffers except for Sp == S.
void launch_fwd_step(Prec prec, int RB, const DevOps &op, const void *S, const void *Sp, void *Sn, bool rows,
                     bool sample, int t, void *y_out, bool y_is_f64, double yscale, hipStream_t s);

// Transpose sweep in the three-level form (Sec. 5.1 eq. (adjoint-verlet) within the
// recursion (backward-recursion), q = M_L^{-1}(v_hat + dt/2 p_hat)).  init: q0 =
// (dt/2m) Pi^T yhat^{N_T}, qm1 = 0.  step: Sn = S + (S - Sp) - (dt/m)(dt K S + B (S - Sp)
// - Pi^T (yhat^{tb+1} + yhat^{tb})/2); last: Sn = the result G^T yhat = (S - Sp) m/dt -
// (dt K S - B Sp - Pi^T yhat^{tb}/2) with tb = 0.  yhat[(t*n_obs + s)*RB + r] * yscale,
// float64 or the sweep type (t = 0 .. N_T - 1 for yhat^1 .. yhat^{N_T}).
void launch_adj_init(Prec prec, int RB, const DevOps &op, void *q0, void *qm1, const void *yhat, bool y_is_f64,
                     double yscale, hipStream_t s);
void launch_adj_step(Prec prec, int RB, const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int tb,
                     const void *yhat, bool y_is_f64, double yscale, hipStream_t s);

// Several meshes' steps in one launch (vector-lane kernels only: RB * sizeof(T) >= 16,
// see multi_step_supported; at most kMaxMeshes meshes).  Each entry is one mesh's
// arguments of launch_fwd_step / launch_adj_step; all share prec, RB and y type.
constexpr int kMaxMeshes = 4;
struct FwdStep {
    const DevOps *op;
    const void *S, *Sp;
    void *Sn;
    bool rows, sample;
    int t;
    void *y;
    double yscale;
};
struct AdjStep {
    const DevOps *op;
    const void *S, *Sp;
    void *Sn;
    bool last;
    int tb;
    const void *yh;
    double yscale;
};
bool multi_step_supported(Prec prec, int RB);
// largest RHS block of the step kernels: a row of the block spans at most one
// wave of 16-byte lanes (256 float32 or 128 float64 values)
int max_rhs_block(Prec prec);
void launch_fwd_multi(Prec prec, int RB, bool y_is_f64, const FwdStep *st, int n, hipStream_t s);
void launch_adj_multi(Prec prec, int RB, bool y_is_f64, const AdjStep *st, int n, hipStream_t s);

// Whittle-Matern spectral prior (pat_spectral.hip): p0 = P w, P = I_h F^* diag(a) F on a
// periodic n^3 grid (G = n^3 points, index (k*n + j)*n + i), I_h trilinear to the nodes.
struct SpecOps {
    int n = 0, logn = 0;
    int64_t G = 0;
    const double *amp = nullptr;                   // a(k) on the half spectrum, [ky][kx < n/2 + 1][kz]
    const double *tw = nullptr;                    // exp(-2 pi i j / n), j < n/2, as (re, im) pairs
    const int32_t *ig = nullptr;                   // [N][8] grid corners of each (internal) node
    const double *iw = nullptr;                    // [N][8] trilinear weights
    const int32_t *tptr = nullptr, *tq = nullptr;  // transpose of I_h by grid point (CSR: nodes)
    const double *tw8 = nullptr;                   // its weights
};
bool spectral_rb_ok(int RB);
// y (mesh [N][RB], float64 or the sweep type) = P x, x latent [G][RB] float64;
// gr [G][RB] and gc [G][RB] complex are work buffers
void launch_spectral(const SpecOps &sp, int RB, const double *x, double *gr, double *gc, Prec out_prec, void *y,
                     int64_t N, hipStream_t s);
// y (latent [G][RB]) = scale * P^T v + add (add may be null); v mesh [N][RB] in in_prec
void launch_spectral_t(const SpecOps &sp, int RB, const void *v, Prec in_prec, double scale, const double *add,
                       double *gr, double *gc, double *y, hipStream_t s);

// Layout conversions.  Node vectors: user [R][N] (rows rb0..rb0+RB-1, zero-padded
// past R) <-> internal [N][RB]; data: user [R][M] <-> internal [M][RB].
void launch_pack(bool in_f64, bool out_f64, const void *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                 const int32_t *perm, void *out, hipStream_t s);
void launch_unpack(bool in_f64, bool out_f64, const void *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                   const int32_t *perm, void *out, hipStream_t s);

// CGLS helpers (all float64 unless noted; [rows][RB] layouts).
void launch_fill(double *x, int64_t count, double v, hipStream_t s);
void launch_cast_to_state(Prec prec, const double *x, void *P, int64_t count, hipStream_t s);
void launch_build_rhs(const double *yobs, const double *eta, int64_t S, int64_t rb0, int RB, int64_t M, double isig,
                      double *bd, hipStream_t s);
// Counter-based standard normals (Philox4x64-10 + Box-Muller): normal j of stream
// (seed, kind, k); kind 0 = eta (j = t*N_obs + s), kind 1 = xi (j = caller node id).
void launch_normals(uint64_t seed, int kind, int64_t k0, int64_t S, int64_t len, double *out, hipStream_t s);
// as launch_build_rhs with eta_{k0+rb0+r} drawn on the fly
void launch_build_rhs_rng(const double *yobs, uint64_t seed, int64_t k0, int64_t S, int64_t rb0, int RB, int64_t M,
                          double isig, double *bd, hipStream_t s);
// xi [N][RB] (internal order) drawn for samples k0+rb0+r, zero past S
void launch_xi_rng(uint64_t seed, int64_t k0, int64_t S, int64_t rb0, int RB, int64_t N, const int32_t *perm,
                   double *xi, hipStream_t s);
void launch_prior(const DevOps &op, int RB, double a, const double *x, double *y, hipStream_t s);
// y = L^T x = M_L^{1/2} x + a K1 (M_L^{-1/2} x)
void launch_prior_t(const DevOps &op, int RB, double a, const double *x, double *y, hipStream_t s);
void launch_gext_t_combine(Prec prec, const DevOps &op, int RB, double a, double isig, const void *PH,
                           const double *rp, double *out, hipStream_t s);
// partial sums: part[b][r] = sum over rows of block b of x*y (y == x gives squares)
constexpr int kDotBlocks = 512;
void launch_dot_partial(const double *x, const double *y, int64_t rows, int RB, double *part, hipStream_t s);
// finalize: mode 0: out[r] = sum partA (+ sum partB if non-null)
void launch_dot_final(const double *partA, const double *partB, int RB, double *out, hipStream_t s);
// part[b][r] = sum over rows of block b of (a[row*lda + aoff + r] - y[row*RB + r])^2, r < RB
// (kDotBlocks partial blocks; finish with launch_dot_final)
void launch_diff_sq_partial(const double *a, int lda, int aoff, const double *y, int64_t rows, int RB, double *part,
                            hipStream_t s);
// out[row*RB + r] = in[row*ldin + c0 + r]: columns [c0, c0 + RB) of a wider block
void launch_cols(const double *in, int ldin, int c0, double *out, int64_t rows, int RB, hipStream_t s);
// scalar stages of CGLS, on device arrays of length RB
void launch_scalar_alpha(const double *gamma, const double *delta, double *alpha, int RB, hipStream_t s);
void launch_scalar_gamma(double *gamma, const double *gnew, double *beta, double *invn, int first, int RB,
                         hipStream_t s);
// hist[(rb0+r)*ld + col] = sqrt(a + b) and diag[2*(that)] = (sqrt(a), sqrt(b)); either may be null
void launch_resid(const double *a, const double *b, double *hist, double *diag, int64_t ld, int64_t col, int64_t rb0,
                  int64_t R, int RB, hipStream_t s);
// x += alpha*d ; rp -= alpha*qp  (N rows)   and   rd -= alpha*qd (M rows)
void launch_update_xr(double *x, const double *d, double *rp, const double *qp, const double *alpha, int64_t rows,
                      int RB, hipStream_t s);
void launch_axpy_neg(double *y, const double *x, const double *alpha, int64_t rows, int RB, hipStream_t s);
// Q[k] = s * invn ; d = s + beta d
void launch_append_dir(const double *sv, double *Qk, double *d, const double *invn, const double *beta, int first,
                       int64_t rows, int RB, hipStream_t s);
// reorthogonalisation: s -= sum_j coef[j] Q[j] (j < k), coef from launch_reorth_coef.  The
// multi-dot streams k basis vectors per call and needs more workgroups than the plain dots
// (4 per CU); its partial sums take kMultiBlocks x 2k x RB doubles.
constexpr int kMultiBlocks = 1024;
void launch_project(const double *Q, double *sv, const double *coef, int k, int64_t rows, int RB, hipStream_t s);
// Both Gram-Schmidt passes' coefficients from one read of the basis Q[0..k-1] (Q[k-1] the
// newest): c1 = Q^T s and the Gram row Q^T Q[k-1] (part: kMultiBlocks x 2k x RB, cg: 2k x RB),
// the row stored into gram [kcap][kcap][RB], then coef = c1 + (c1 - gram c1) (k x RB).
void launch_reorth_coef(const double *Q, const double *sv, int k, int64_t rows, int RB, double *part, double *cg,
                        double *gram, int kcap, double *coef, hipStream_t s);
// LSQR scalar recurrences (device arrays of length RB each).
struct LsqrScalars {
    double *alpha, *beta, *alpha1, *beta1, *rhob, *phib, *cs, *sn, *rho, *zfac, *step, *inv;
};
// InitBeta:  beta_1 = sqrt(n1 + n2), inv = 1/beta_1
// InitAlpha: alpha_1 = sqrt(n1), inv = 1/alpha_1, phi_bar = beta_1, rho_bar = alpha_1
// Beta:      beta_{k+1} = sqrt(n1 + n2), inv = 1/beta, rotation (rho, c, s), phi_bar, step = phi/rho
// Alpha:     alpha_{k+1} = sqrt(n1), inv = 1/alpha, rho_bar = -c alpha, zfac = s alpha / rho
enum class LsqrStage : int { InitBeta, InitAlpha, Beta, Alpha };
void launch_lsqr_scalar(LsqrStage st, const LsqrScalars &c, const double *n1, const double *n2, int RB,
                        hipStream_t s);
// out = sa*ca[r]*a + sb*cb[r]*b (null ca/cb: 1; null b: no second term); out may alias a or b
void launch_lincomb(double *out, const double *a, const double *ca, double sa, const double *b, const double *cb,
                    double sb, int64_t rows, int RB, hipStream_t s);
// v = inv*sv ; w = v - zfac*w (first: w = v) ; Qk = v if non-null
void launch_lsqr_vw(const double *sv, const double *inv, const double *zfac, double *v, double *w, double *Qk,
                    int first, int64_t rows, int RB, hipStream_t s);
// diagnostics of diag [S][n_it][2] (see pat_solver_diagnostics); outputs may be null
void launch_diagnostics(const double *diag, int64_t S, int n_it, int64_t n_data, double tau, double *data,
                        double *prior, double *ext, int32_t *first, hipStream_t s);
// pointwise mean and std (1/(S-1)) of samples [S][N]
void launch_stats(const double *samples, int64_t S, int64_t N, double *mean, double *std, hipStream_t s);

}  // namespace pat
