/*
 * pat.h -- C ABI of libpat, the MI355X (gfx950) implementation of the
 * matrix-free randomize-then-optimize (RTO) posterior sampler for 3D
 * photoacoustic tomography of "3D Uncertainty Quantification for
 * Photoacoustic Tomography" (arXiv 2607.21373).
 *
 * Conventions for every entry point:
 *  - Device buffers are plain device pointers owned by the caller (for example
 *    PyTorch allocations).  The library never frees them and never keeps them
 *    beyond the call's stream order.  Host arrays in pat_problem_desc are copied
 *    during pat_problem_create.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *    device work is enqueued on it; results are ready when the stream has reached
 *    the point of the call.  Calls return without waiting for the device, except
 *    those whose comment says that they synchronise (rto_sample,
 *    rto_sample_batch, the autotuners, pat_spectral_prior_set, pat_sync).
 *  - Node-indexed vectors use the caller's node numbering (the library reorders
 *    nodes internally and converts at the boundary).
 *  - Errors: validation failures return a negative pat_status before any device
 *    work is enqueued and leave outputs untouched.  pat_last_error() returns a
 *    thread-local message for the last failing call on the calling thread.
 *    Asynchronous device faults surface at a later call or at pat_sync().
 *  - A handle is not thread-safe; distinct handles are independent.  Device work
 *    enqueued through one handle must not overlap in time on different streams:
 *    it shares the handle's sweep buffers.
 */
#ifndef PAT_H
#define PAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PAT_OK = 0,
    PAT_ERR_INVALID_ARG = -1,   /* bad sizes, NULL pointers, ids out of range, sensor outside the mesh */
    PAT_ERR_UNSTABLE_DT = -2,   /* dt fails the stability check at create */
    PAT_ERR_NONFINITE = -3,     /* non-finite input or a non-finite CGLS scalar */
    PAT_ERR_OUT_OF_MEMORY = -4, /* host or device allocation failed */
    PAT_ERR_HIP = -5,           /* a HIP runtime call failed (including: no device) */
    PAT_ERR_INTERNAL = -6
} pat_status;

typedef enum {
    PAT_F64 = 0,  /* float64 state and matrices */
    PAT_F32 = 1   /* float32 state and matrices */
} pat_precision;

typedef struct pat_problem pat_problem;

/* Discrete problem of Sec. 3 (P1 tetrahedra, lumped mass, Stormer-Verlet). */
typedef struct {
    int32_t n_nodes;            /* N */
    const double *coords;       /* host [N][3] node coordinates */
    int64_t n_tets;             /* E */
    const int32_t *tets;        /* host [E][4] node ids of each tetrahedron */
    const double *c_tet;        /* host [E] wave speed per tetrahedron, or NULL for c = 1 */
    int32_t absorbing;          /* 1: first-order absorbing boundary (Sec. 2 eq. (boundary)), 0: reflecting */
    int32_t n_obs;              /* number of sensors */
    const int32_t *sensor_nodes;/* host [n_obs] node ids (sensors at nodes, Sec. 3 eq. (lagrange)), or NULL */
    const double *sensor_pos;   /* host [n_obs][3] sensor points (P1 interpolation in the containing tet), or NULL */
    double dt;                  /* time step */
    int32_t n_steps;            /* N_T: data at t_n = n dt, n = 1..N_T */
    int32_t device;             /* HIP device ordinal, -1 = current device */
    int32_t check_dt;           /* 1: reject dt that fails the stability check, 0: skip the check */
} pat_problem_desc;

typedef struct {
    int32_t n_nodes, n_obs, n_steps;
    int64_t n_tets, nnz_k, nnz_b;
    int32_t n_boundary_nodes, max_row_nnz;
    double dt, lambda_max;      /* lambda_max: estimate of the largest eigenvalue of M_L^{-1} K */
    int64_t device_bytes;       /* device memory held by the handle (matrices + workspaces) */
    int64_t b_stored;           /* stored boundary-mass values (full stiffness rows of boundary nodes) */
} pat_problem_info;

/* Sweep timing of rto_sample, from HIP events recorded on the caller's stream
 * around each N_T-step sweep (forward: N_T step launches + 1 sampling launch;
 * transpose: 1 init launch + N_T step launches). */
typedef struct {
    double fwd_ms, adj_ms;      /* summed sweep durations */
    int64_t fwd_sweeps, adj_sweeps;
} pat_profile;

/* Assemble K (c^2 stiffness), K1 (unit-coefficient stiffness), the lumped mass
 * M_L = diag(M 1) and the consistent boundary mass B of Sec. 3 (matrices below
 * eq. (semi-discrete)); locate the sensors; check dt; upload to the device.
 * Exactly one of sensor_nodes / sensor_pos must be given.  On success *out owns
 * the device copies; release with pat_problem_destroy. */
pat_status pat_problem_create(const pat_problem_desc *desc, pat_problem **out);
pat_status pat_problem_destroy(pat_problem *p);
pat_status pat_problem_get_info(const pat_problem *p, pat_problem_info *out);

/* Forward map Y = G p0 of Sec. 3 eq. (discrete-wave-matrix): z0 = (p0, 0),
 * z^n = A_dt^n z0, Y[n-1][s] = (Pi z^n)_s for n = 1..N_T.
 *   p0 device [R][N], y device [R][N_T][N_obs]; both of type `prec`. */
pat_status pat_forward(pat_problem *p, int64_t R, const void *p0, void *y, pat_precision prec, void *stream);

/* pat_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * layouts and result as pat_forward; the device work is launched directly on
 * `stream` (no graph of its own, so a caller may capture it), and the sweep state
 * and data staging live in a fixed device scratch array of 64 MiB per device
 * (held from the library's first use on a device until the process ends).  No
 * hipMalloc, hipFree or other allocating call is made.  Right-hand sides run in
 * blocks of the largest power of two <= pat_forward's block whose state and
 * staging, (3 N + N_T N_obs) x block x element size, fit the scratch; a problem
 * for which one right-hand side does not fit is PAT_ERR_INVALID_ARG.  All calls
 * on one device share its scratch: calls that overlap in time on one device (on
 * different streams or threads) race and give undefined results.  Nothing in the
 * scratch needs to start at zero: each block overwrites what it reads. */
pat_status pat_forward_noalloc(pat_problem *p, int64_t R, const void *p0, void *y, pat_precision prec, void *stream);

/* Transpose map p = G^T yhat of Sec. 5.1 eqs. (transpose-definition),
 * (backward-recursion) and (adjoint-verlet): exact transpose of pat_forward in
 * exact arithmetic.  yhat device [R][N_T][N_obs], p device [R][N]; type `prec`. */
pat_status pat_adjoint(pat_problem *p, int64_t R, const void *yhat, void *p_out, pat_precision prec, void *stream);

/* Prior factor L = M_L^{-1/2}(M_L + a K1) (transpose = 0) or its transpose
 * L^T = (M_L + a K1) M_L^{-1/2} (transpose = 1), so L^T L is the prior precision;
 * a = 0 gives M_L^{1/2}, the square root of the precision of eq. (iid-prior).
 *   x, y device [R][N] float64 (caller numbering); y must not alias x. */
pat_status pat_prior_apply(pat_problem *p, int64_t R, double prior_a, int transpose, const double *x, double *y,
                           void *stream);

/* Least-squares solver of each RTO sample (Sec. 5, Algorithm 1, App. A). */
typedef enum {
    PAT_CGLS = 0, /* CG on the normal equations; reorth acts on the normalised residuals s_j = G_ext^T r_j */
    PAT_LSQR = 1  /* Paige-Saunders Golub-Kahan bidiagonalisation; reorth acts on the right vectors v_j */
} pat_solver;

/* Prior of the RTO sampler. */
typedef enum {
    PAT_PRIOR_FE = 0,       /* the FE prior factor L = M_L^{-1/2}(M_L + a K1) (prior_a) on the nodal values */
    PAT_PRIOR_SPECTRAL = 1  /* the Whittle-Matern spectral prior set with pat_spectral_prior_set; the solve runs
                               in its latent space (Sec. 6.4) */
} pat_prior_kind;

/* Parameters of the RTO sampler (Sec. 5 eq. (optimization), Algorithm 1). */
typedef struct {
    double sigma;              /* noise standard deviation (> 0) */
    double prior_a;            /* prior factor L = M_L^{-1/2}(M_L + a K1); a = 0 gives M_L^{1/2}, eq. (iid-prior) */
    int32_t n_iter;            /* solver iterations (fixed; >= 1) */
    int32_t reorth;            /* 1: full reorthogonalisation (default); see pat_solver */
    pat_precision sweep_prec;  /* precision of the wave sweeps; solver vectors and scalars are always float64 */
    int32_t rhs_block;         /* samples per multi-RHS block: a power of two up to 256 (float32 sweeps) or 128
                                  (float64 sweeps; a row of the block spans at most one wave), or 0 = the
                                  autotuned block for (S, sweep_prec) if pat_autotune / pat_batch_autotune
                                  ran, else the smallest power of two >= S (at most 64).  One block's
                                  sweep state, N x block x element size, must stay below 4 GiB: automatic
                                  choices halve the block until it does, an explicit larger block is
                                  PAT_ERR_INVALID_ARG */
    const double *eta;         /* device [S][N_T][N_obs] standard-normal data perturbations, or NULL */
    const double *xi;          /* device [S][N] standard-normal prior perturbations, or NULL (both or neither) */
    int32_t solver;            /* pat_solver; 0 (CGLS) when the struct is zero-initialised */
    double *diag_hist;         /* device [S][n_iter+1][2] float64 or NULL: per iteration the data and prior parts
                                  (||y_obs/sigma + eta - G p/sigma||, ||xi - L p||) of the residual */
    uint64_t seed;             /* eta == xi == NULL: the sampler draws them itself, see pat_draw_normals */
    int64_t sample0;           /* stream index of the first sample (disjoint ranges give independent samples) */
    int32_t prior;             /* pat_prior_kind; 0 (FE) when the struct is zero-initialised.  With
                                  PAT_PRIOR_SPECTRAL, xi is device [S][n^3] (latent white noise, grid order),
                                  prior_a is ignored, the unknown of each solve is the latent vector w and the
                                  samples are p0 = P w */
    double *latent;            /* PAT_PRIOR_SPECTRAL: device [S][n^3] latent samples w, or NULL */
    double *final_resid;       /* device [S] float64 or NULL: ||b_k - G_ext p_k||_2 of each returned sample
                                  (Sec. 5 eq. (lsqr-residual)), recomputed after the solve from p_k with a
                                  float64 forward sweep and the float64 prior factor, whatever sweep_prec
                                  (resid_hist holds the residual the solver carries instead).  Costs one
                                  float64 forward sweep per RHS block (per 128 RHS of wider blocks) */
} pat_rto_params;

/* S posterior samples by RTO.  Sample k solves
 *   min_p || G_ext p - b_k ||_2,  G_ext = [G/sigma ; L],  b_k = [y_obs/sigma + eta_k ; xi_k]
 * (eq. (extended-matrices) with p_prior = L^{-1} xi_k) by CGLS or LSQR from p = 0.
 * In exact arithmetic both solvers, with reorthogonalisation, give the same iterates.
 *   y_obs       device [N_T][N_obs] float64
 *   samples     device [S][N] float64 (required)
 *   mean, std   device [N] float64 or NULL: pointwise mean and standard deviation
 *               with 1/(S-1) normalisation (eq. (ergodic)); std needs S >= 2
 *   resid_hist  device [S][n_iter+1] float64 or NULL: ||b_k - G_ext p_k^{(j)}||_2 per iteration, as
 *               carried by the solver's recurrences
 * Scratch memory is owned by the handle and grows to the largest block seen.
 * Synchronises `stream` before it returns: it reads back one per-sample solver
 * scalar (CGLS gamma, LSQR phi_bar) to report a breakdown.  PAT_ERR_NONFINITE
 * then comes after every output has been written (the non-finite samples included). */
pat_status rto_sample(pat_problem *p, const double *y_obs, const pat_rto_params *prm, int64_t S,
                      double *samples, double *mean, double *std, double *resid_hist, void *stream);

/* Convergence diagnostics of Sec. 6.1 from a diag_hist of rto_sample (the normalised data
 * misfit, prior contribution and extended residual per iteration, and the discrepancy
 * principle).  diag: device [S][n_iter+1][2] float64, (||r_d||, ||r_p||) per iteration with
 * r_d = y_obs/sigma + eta - G p/sigma (the whitened data residual) and r_p = xi - L p.
 * n_data = N_T N_obs.  Outputs (device, each may be NULL):
 *   data  [S][n_iter+1] float64: ||r_d|| / sqrt(n_data)  (1 at the discrepancy level sigma sqrt(N_T N_obs))
 *   prior [S][n_iter+1] float64: ||r_p|| / ||b||, ||b|| the extended residual at iteration 0 (x = 0)
 *   ext   [S][n_iter+1] float64: sqrt(||r_d||^2 + ||r_p||^2) / ||b||
 *   first [S] int32: the first iteration j with ||r_d|| <= tau sqrt(n_data), or -1 if none
 * A zero ||b|| leaves the ratios unscaled.  Runs on the current device; asynchronous. */
pat_status pat_solver_diagnostics(const double *diag, int64_t S, int32_t n_iter, int64_t n_data, double tau,
                                  double *data, double *prior, double *ext, int32_t *first, void *stream);

/* Whittle-Matern prior of Sec. 4.1.2 eq. (matern-cov-op), built as in Sec. 6.4: a
 * latent white-noise vector w on a periodic grid of n^3 points over the cube
 * [lo, lo + side)^3 (index (k*n + j)*n + i for the point lo + h (i, j, k), h = side/n)
 * gives the field u = F^* diag(a) F w, F the unitary 3D DFT and
 * a(k) = c (ell^-2 + |k|^2)^(-expo/2), expo = nu + d/2 (3 for the paper's s = 1.5),
 * c chosen so that the pointwise variance of u is sigma^2.  Trilinear
 * interpolation I_h to the mesh nodes gives p0 = P w, P = I_h F^* diag(a) F. */
typedef struct {
    int32_t n;       /* grid points per axis: a power of two in [8, 128] */
    double lo[3];    /* box corner */
    double side;     /* box side; every mesh node must satisfy lo <= x < lo + side */
    double ell;      /* correlation length */
    double sigma;    /* marginal standard deviation */
    double expo;     /* covariance exponent nu + d/2 */
} pat_spectral_desc;

/* Set (or, with d == NULL, clear) the handle's spectral prior; replaces any earlier one
 * and frees the latent-space workspaces.  Synchronises the device. */
pat_status pat_spectral_prior_set(pat_problem *p, const pat_spectral_desc *d);

/* transpose = 0: y = P x, x device [R][n^3] -> y device [R][N];
 * transpose = 1: y = P^T x, x device [R][N] -> y device [R][n^3].  float64. */
pat_status pat_spectral_apply(pat_problem *p, int64_t R, int transpose, const double *x, double *y, void *stream);

/* Autotuner of the RHS block.  With B the smallest power of two >= S (at most 256
 * for float32 and 128 for float64 sweeps), for each candidate block RB (powers of
 * two from max(1, min(B, 64) / 16) up to B) it times 8 forward and 8
 * transpose steps, captured in graphs as the sweeps are, with HIP events after a
 * warm-up, prices S samples as
 * ceil(S/RB) * (forward + transpose step) and records the cheapest RB for
 * (S, prec) in the handle, where rto_sample's rhs_block = 0 finds it.
 *   rhs_block  host int32 or NULL: the chosen block
 *   step_us    host double or NULL: its priced cost of one forward plus one
 *              transpose step for all S samples, in microseconds
 * Synchronises `stream`.  The sweep workspaces it allocates for candidate blocks
 * other than the chosen one are freed again (those that existed before are kept,
 * with their contents overwritten). */
pat_status pat_autotune(pat_problem *p, int64_t S, pat_precision prec, int32_t *rhs_block, double *step_us,
                        void *stream);

/* Several problems sampled together ("uneven batch"): their forward and transpose
 * sweeps run as one launch per time step over the row tiles of all meshes (a
 * workgroup finds its mesh from the running tile counts), while each keeps its own
 * solver state.  Needs the same device and the same number of time steps; at
 * most 4 problems, each at most once.  The problems must outlive the batch.  One
 * launch per step covers all meshes when RB * sizeof(sweep type) >= 16 bytes;
 * smaller blocks launch per mesh within the same step. */
typedef struct pat_batch pat_batch;
pat_status pat_batch_create(pat_problem *const *problems, int32_t n, pat_batch **out);
pat_status pat_batch_destroy(pat_batch *b);

/* pat_autotune for the batch (S = the largest per-problem sample count).  For each
 * candidate block it also times, per direction (forward, transpose), the three
 * launch modes of pat_batch_merge and keeps the fastest; rto_sample_batch uses
 * these choices when rhs_block is 0 or equals the tuned block (otherwise it merges). */
pat_status pat_batch_autotune(pat_batch *b, int64_t S, pat_precision prec, int32_t *rhs_block, double *step_us,
                              void *stream);

/* Launch mode of rto_sample_batch per sweep direction: 1 = one merged launch per
 * time step for all problems; 0 = one launch per problem within each time step;
 * 2 = each problem's whole sweep in turn (keeps a small mesh's working set in
 * cache across its steps); -1 = the autotuned choice (merged when not tuned).
 * Results do not depend on it. */
pat_status pat_batch_merge(pat_batch *b, int32_t forward, int32_t transpose);

/* rto_sample for every problem m of the batch at once: arrays of n entries
 * (n = problems in the batch).  prm[m] gives problem m's sigma, prior_a,
 * perturbations (eta, xi or seed, sample0), diag_hist and final_resid; n_iter, reorth,
 * sweep_prec, rhs_block and solver must agree across m.  All problems use one RHS
 * block; with unequal S the smaller ones run zero right-hand sides in the later
 * blocks.  mean, std, resid_hist: arrays or NULL, entries may be NULL.  Results
 * equal rto_sample on each problem alone.  Synchronises `stream` before it returns,
 * and reports PAT_ERR_NONFINITE as rto_sample does (outputs already written). */
pat_status rto_sample_batch(pat_batch *b, const double *const *y_obs, const pat_rto_params *prm, const int64_t *S,
                            double *const *samples, double *const *mean, double *const *std,
                            double *const *resid_hist, void *stream);

/* Standard normals of the sampler's own perturbations (Algorithm 1 draws eta_k and
 * xi_k): out[s][j] = normal j of stream (seed, kind, k0 + s), s < S, j < len,
 * device float64 [S][len].  kind 0 is eta (j = t*N_obs + sensor), kind 1 is xi
 * (j = node id in the caller's numbering); rto_sample with eta == xi == NULL uses
 * streams (seed, kind, sample0 + k) for its sample k.  Normal j is lane j%4 of
 * the Philox4x64-10 block (Salmon, Moraes, Dror and Shaw, SC'11) with counter
 * (j/4, k, kind, 0) and key (seed, 0); lanes (0,1) and (2,3) are Box-Muller pairs
 * with u1 = 1 - U(first word), u2 = U(second word), U(w) = (w >> 11) 2^-53.
 * Runs on the current device; kind must be 0 or 1. */
pat_status pat_draw_normals(uint64_t seed, int32_t kind, int64_t k0, int64_t S, int64_t len, double *out,
                            void *stream);

/* Host-only view of the setup (no device is touched): runs the validation and
 * assembly of pat_problem_create and copies the assembled operators out in the
 * caller's node numbering.  Call once with rowptr == NULL to get the sizes in
 * *nnz_out (entries of the stiffness pattern); then pass
 *   rowptr [N+1], col [nnz], kval [nnz] (K), k1val [nnz] (K1), bval [nnz] (B on
 *   the same pattern, zero off the boundary), mass [N] (M_L), snode [n_obs][4],
 *   sw [n_obs][4] (sensor interpolation nodes and weights), lambda_max [1].
 * For tests and diagnostics; returns the same status pat_problem_create would
 * return for the descriptor up to the device steps. */
pat_status pat_host_assemble(const pat_problem_desc *desc, int64_t *nnz_out, int32_t *rowptr, int32_t *col,
                             double *kval, double *k1val, double *bval, double *mass, int32_t *snode, double *sw,
                             double *lambda_max);

/* Enable (1) or disable (0) sweep timing in rto_sample; enabling resets the counters. */
pat_status pat_profile_enable(pat_problem *p, int enable);
pat_status pat_profile_get(const pat_problem *p, pat_profile *out);

/* Wait for all work of the handle's device, report asynchronous errors. */
pat_status pat_sync(pat_problem *p);

/* Thread-local description of the last error ("" if none). */
const char *pat_last_error(void);

/* Library version string. */
const char *pat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PAT_H */
