// HIP kernels of libpat for gfx950 (MI355X, CDNA4, wave64).
//
// Data layout: a block of RB right-hand sides is stored node-major with the RHS
// fastest, x[i*RB + r], so the RB values a row gathers from one neighbour are
// one contiguous RB*sizeof(T) segment.  Blocks of at least 16 bytes per row use
// the vector-lane kernels (16 bytes per lane, further down).  Below that (one
// RHS, or two floats) the scalar-lane kernels split a row's padded slots over
// 4 lanes per RHS and combine their sums with cross-lane shuffles.
//
// Paper: "3D Uncertainty Quantification for Photoacoustic Tomography"
// (arXiv 2607.21373).  The time stepping is Sec. 3 eq. (fully-discrete) with
// M replaced by M_L; the transposed stepping is Sec. 5.1 eq. (adjoint-verlet)
// with the recursion (backward-recursion).
//
// Both are carried as three-level recurrences in one state vector, so that a
// step reads two state vectors and writes one (the velocity form reads two and
// writes two).  Forward: with S^n = p^{n+1/2} (p^{1/2} = p^0 since v^0 = 0),
// the three substeps give dt v^n = S^n - S^{n-1} and
//   S^{n+1} = S^n + (S^n - S^{n-1}) - (dt/m) (dt K S^n + B (S^n - S^{n-1})),
//   p^n = (S^{n-1} + S^n) / 2  (the sampled pressure),
// started from S^{-1} = S^0 = p^0.  Transposed: write inj_j = Pi^T yhat^{N_T - j}
// and q_k = M_L^{-1}(v_hat + dt/2 p_hat) after k transposed steps.  Then
// p_hat_{k+1} = (q_{k+1} - q_k) m/dt + B q_k + inj_{k+1}/2, and eliminating p_hat
// leaves the same recurrence for q with a source:
//   q_{k+1} = q_k + (q_k - q_{k-1}) - (dt/m) (dt K q_k + B (q_k - q_{k-1}) - (inj_k + inj_{k+1})/2)
// for k = 0 .. N_T - 2, started from q_{-1} = 0, q_0 = (dt/2m) inj_0; the result is
//   G^T yhat = (q_K - q_{K-1}) m/dt - (dt K q_K - B q_{K-1} - inj_K/2),  K = N_T - 1.
// In exact arithmetic both forms give the same maps.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pat_internal.h"
#include "pat_kernels.h"
#include "pat_tiles.h"

namespace pat {
namespace {

__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int RB>
struct Geo {
    static constexpr int SPLIT = RB >= 8 ? 1 : RB == 1 ? 4 : 8 / RB;  // lanes sharing one RHS of a row
    static constexpr int LPR = RB * SPLIT;              // lanes per row
    static constexpr int RPW = 64 / LPR;                // rows per wave
    static constexpr int RPB = 4 * RPW;                 // rows per 256-thread workgroup
    static constexpr int W = 16;                        // padded slots per row (HostProblem::kEll)
    static constexpr int PER = W / SPLIT;               // padded slots per lane
};

template <int RB, int LPR>
__device__ __forceinline__ float lane_sum(float v) {
    for (int o = RB; o < LPR; o <<= 1) v += __shfl_xor(v, o);
    return v;
}
template <int RB, int LPR>
__device__ __forceinline__ double lane_sum(double v) {
    for (int o = RB; o < LPR; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Row operands of the padded layout (see HostProblem::kEll): slot j < 16 of row i
// at i*16 + j, the entries beyond 16 in (xptr, xcol, xval), and for boundary rows
// the B value of each slot at bslot[bsoff[i] + slot].
template <typename T>
struct RowOps {
    const int32_t *ecol, *xptr, *xcol, *bsoff;
    const T *eval, *xval, *bslot, *dtm;
    const int32_t *bnum;  // boundary rows: slots with a nonzero B come first, bnum of them
};

// Operands of one row as seen by one lane: its padded slots' columns and
// weights, the boundary-slot offset, the overflow range and dt/m.
template <typename T, int RB>
struct RowMeta {
    int c[Geo<RB>::PER];
    T w[Geo<RB>::PER];
    int bo, x0, x1;
    T dm;
};

template <typename T, int RB>
__device__ __forceinline__ void load_meta(const RowOps<T> &o, int row, int part, RowMeta<T, RB> &m) {
    using G = Geo<RB>;
    const int64_t eb = int64_t(row) * G::W;
#pragma unroll
    for (int j = 0; j < G::PER; ++j) {
        m.c[j] = o.ecol[eb + part + j * G::SPLIT];
        m.w[j] = o.eval[eb + part + j * G::SPLIT];
    }
    m.bo = o.bsoff[row];
    m.x0 = o.xptr[row];
    m.x1 = o.xptr[row + 1];
    m.dm = o.dtm[row];
}

// The value a boundary slot multiplies: S - S_prev in a step, -S_prev in the
// transpose sweep's closing launch (only_prev).
template <typename T>
__device__ __forceinline__ T bdiff(T x, T y, bool only_prev) { return only_prev ? -y : x - y; }

// One row of a three-level step: S' = S + ((S - Sp) - (dt/m)(dt K S + B (S - Sp) - src))
// from acc = (K S)_row, bacc = (B (S - Sp))_row and the source src (0 forward).
template <typename T>
__device__ __forceinline__ T step_update(T cur, T prev, T acc, T bacc, T src, T dm, T dt) {
    const T f = mad(dt, acc, bacc) - src;
    return cur + mad(-dm, f, cur - prev);
}
// The transpose sweep's result, (q - q_prev) m/dt - (dt K q - B q_prev - src), from
// acc = (K q)_row and bacc = -(B q_prev)_row.
template <typename T>
__device__ __forceinline__ T adj_result(T cur, T prev, T acc, T bacc, T src, T dm, T dt) {
    const T f = mad(dt, acc, bacc) - src;
    return (cur - prev) / dm - f;
}

// acc = sum over the row's entries of K(row, k) X[col_k][r], and for a boundary row
// bacc = sum of B(row, k) bdiff(X[col_k][r], Y[col_k][r]).  All PER gathers of the
// lane are issued before any is consumed; sums run in slot order, then the entries
// beyond 16.
template <typename T, int RB>
__device__ __forceinline__ void row_sums(const RowOps<T> &o, const RowMeta<T, RB> &m, int part, int r,
                                         const T *__restrict__ X, const T *__restrict__ Y, bool with_b,
                                         bool only_prev, T &acc, T &bacc) {
    using G = Geo<RB>;
    T x[G::PER];
#pragma unroll
    for (int j = 0; j < G::PER; ++j) x[j] = X[int64_t(m.c[j]) * RB + r];
#pragma unroll
    for (int j = 0; j < G::PER; ++j) acc = mad(m.w[j], x[j], acc);
    if (with_b) {
        const T *Bv = o.bslot + m.bo;
        T bw[G::PER], y[G::PER];
#pragma unroll
        for (int j = 0; j < G::PER; ++j) bw[j] = Bv[part + j * G::SPLIT];
#pragma unroll
        for (int j = 0; j < G::PER; ++j) y[j] = Y[int64_t(m.c[j]) * RB + r];
#pragma unroll
        for (int j = 0; j < G::PER; ++j) bacc = mad(bw[j], bdiff(x[j], y[j], only_prev), bacc);
    }
    for (int k = m.x0 + part; k < m.x1; k += G::SPLIT) {
        const int64_t cj = int64_t(o.xcol[k]) * RB + r;
        const T xv = X[cj];
        acc = mad(o.xval[k], xv, acc);
        if (with_b) bacc = mad(o.bslot[m.bo + G::W + (k - m.x0)], bdiff(xv, Y[cj], only_prev), bacc);
    }
}

template <typename T>
struct FwdArgs {
    RowOps<T> o;
    const int32_t *snode;
    const T *sw;
    const T *S, *Sp;  // S^n, S^{n-1}
    T *Sn;            // S^{n+1}
    void *y;
    double yscale;
    int n, n_obs, n_tiles, n_samp, sample, t;
    T dt;
};

// Forward step S^{n+1} = S^n + (S^n - S^{n-1}) - (dt/m)(dt K S^n + B (S^n - S^{n-1})),
// the three-substep Stormer-Verlet update with lumped mass in S^n = p^{n+1/2}.  One
// tile of RPB rows per workgroup; the sampling blocks placed among them write the
// samples y = Pi p^n = Pi (S^n + S^{n-1})/2 of the incoming state, one (sensor, RHS)
// pair per thread.
template <typename T, typename OT, int RB>
__global__ void __launch_bounds__(256) k_fwd(const FwdArgs<T> a) {
    using G = Geo<RB>;
    const int tile = fwd_work(xcd_tile(blockIdx.x, gridDim.x), a.n_tiles, a.n_samp);
    if (tile < a.n_tiles) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int part = (lane / RB) % G::SPLIT, r = lane % RB;
        const int row = tile * G::RPB + wave * G::RPW + lane / G::LPR;
        if (row >= a.n) return;
        RowMeta<T, RB> m;
        load_meta<T, RB>(a.o, row, part, m);
        const int64_t id = int64_t(row) * RB + r;
        T acc = T(0), bacc = T(0);
        row_sums<T, RB>(a.o, m, part, r, a.S, a.Sp, m.bo >= 0, false, acc, bacc);
        acc = lane_sum<RB, G::LPR>(acc);
        bacc = lane_sum<RB, G::LPR>(bacc);
        if (part == 0) a.Sn[id] = step_update(a.S[id], a.Sp[id], acc, bacc, T(0), m.dm, a.dt);
        return;
    }
    const int64_t e = int64_t(tile - a.n_tiles) * 256 + threadIdx.x;
    if (e >= int64_t(a.n_obs) * RB) return;
    const int s = int(e / RB), r = int(e % RB);
    T y = T(0);
    for (int k = 0; k < 4; ++k) {
        const int64_t id = int64_t(a.snode[4 * s + k]) * RB + r;
        y = mad(a.sw[4 * s + k], T(0.5) * (a.S[id] + a.Sp[id]), y);
    }
    OT *yo = static_cast<OT *>(a.y);
    yo[(int64_t(a.t) * a.n_obs + s) * RB + r] = static_cast<OT>(static_cast<double>(y) * a.yscale);
}

template <typename T>
struct AdjArgs {
    RowOps<T> o;
    const int32_t *injptr, *injs;
    const T *injw;
    const T *S, *Sp;  // q_k, q_{k-1}
    T *Sn;            // q_{k+1}, or the result after the last step
    const void *yh;
    double yscale;
    int n, n_obs, n_tiles, last;
    int ta, tb;  // sources: Pi^T yhat at sample indices ta (if >= 0) and tb
    T dt;
};

// Rows with sensor weights are few (four per sensor at most): one wave-uniform
// test of the injection range of the wave's rows [r0, r0 + nrows) lets waves
// without any skip the per-row range loads.
__device__ __forceinline__ bool wave_injects(const int32_t *injptr, int r0, int nrows, int n) {
    const int w0 = __builtin_amdgcn_readfirstlane(r0);
    if (w0 >= n) return false;
    const int w1 = w0 + nrows < n ? w0 + nrows : n;
    return injptr[w0] != injptr[w1];
}

// (Pi^T (yhat^{ta} + yhat^{tb}))_row for RHS r over the row's injection entries
// [e0, e1) (yhat^{ta} left out for ta < 0)
template <typename T, typename YT, int RB>
__device__ __forceinline__ T inject_range(const AdjArgs<T> &a, int e0, int e1, int r) {
    const YT *yh = static_cast<const YT *>(a.yh);
    T inj = T(0);
    for (int e = e0; e < e1; ++e) {
        const int s = a.injs[e];
        T v = static_cast<T>(static_cast<double>(yh[(int64_t(a.tb) * a.n_obs + s) * RB + r]) * a.yscale);
        if (a.ta >= 0) v = static_cast<T>(static_cast<double>(yh[(int64_t(a.ta) * a.n_obs + s) * RB + r]) * a.yscale) + v;
        inj = mad(a.injw[e], v, inj);
    }
    return inj;
}
template <typename T, typename YT, int RB>
__device__ __forceinline__ T inject(const AdjArgs<T> &a, int row, int r) {
    return inject_range<T, YT, RB>(a, a.injptr[row], a.injptr[row + 1], r);
}

// Transposed step q_{k+1} = q_k + (q_k - q_{k-1}) - (dt/m)(dt K q_k + B (q_k - q_{k-1})
// - inj/2), inj = Pi^T (yhat^{ta} + yhat^{tb}); with `last`, the result
// (q_k - q_{k-1}) m/dt - (dt K q_k - B q_{k-1} - inj/2), inj = Pi^T yhat^{tb}.
// One tile of RPB rows per workgroup, each XCD's range walked from its end
// (xcd_tile_rev).  The injection range is loaded with the row operands, a round
// trip earlier than after the sums.
template <typename T, typename YT, int RB>
__global__ void __launch_bounds__(256) k_adj(const AdjArgs<T> a) {
    using G = Geo<RB>;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int part = (lane / RB) % G::SPLIT, r = lane % RB;
    const int wrow0 = xcd_tile_rev(blockIdx.x, gridDim.x) * G::RPB + wave * G::RPW;
    const bool winj = wave_injects(a.injptr, wrow0, G::RPW, a.n);
    const int row = wrow0 + lane / G::LPR;
    if (row >= a.n) return;
    RowMeta<T, RB> m;
    load_meta<T, RB>(a.o, row, part, m);
    int e0 = 0, e1 = 0;
    if (winj) {
        e0 = a.injptr[row];
        e1 = a.injptr[row + 1];
    }
    const int64_t id = int64_t(row) * RB + r;
    T kq = T(0), bq = T(0);
    row_sums<T, RB>(a.o, m, part, r, a.S, a.Sp, m.bo >= 0, a.last, kq, bq);
    kq = lane_sum<RB, G::LPR>(kq);
    bq = lane_sum<RB, G::LPR>(bq);
    if (part == 0) {
        const T cur = a.S[id], prev = a.Sp[id];
        const T src = winj ? T(0.5) * inject_range<T, YT, RB>(a, e0, e1, r) : T(0);
        a.Sn[id] = a.last ? adj_result(cur, prev, kq, bq, src, m.dm, a.dt)
                          : step_update(cur, prev, kq, bq, src, m.dm, a.dt);
    }
}

// ---------------------------------------------------------------------------
// Vector-lane step kernels (used when a row of the RHS block is >= 16 bytes).
//
// Each lane moves 16 bytes (VEC = 4 floats or 2 doubles, i.e. VEC right-hand
// sides), a lane group of LPR = RB / VEC lanes owns one row, and one wave64
// instruction gathers 64/LPR neighbour rows at once.  The padded row operands
// of a tile (column, stiffness and boundary weight per slot, dt/m, overflow
// range) are staged in LDS once per tile and read back as LDS broadcasts.
// ---------------------------------------------------------------------------

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using t = float __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using t = double __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

// Gathers in flight per lane before they are consumed.
constexpr int kGatherChunk = 8;
// Waves per SIMD the register allocation of the step kernels must allow: 8 for
// float32 state, 5 for float64; capped by what the tile's LDS image allows
// (160 KiB per CU; one 4-wave workgroup per tile, one wave per SIMD).
template <typename T, int RB, typename Ops>
constexpr int vwaves() {
    const int want = sizeof(T) == 4 ? 8 : 5;
    const int lds = int(163840 / sizeof(Ops));
    return want < lds ? want : (lds > 0 ? lds : 1);
}
#define PAT_VOCC(T, RB) __attribute__((amdgpu_waves_per_eu(vwaves<T, RB, TileOps<T, RB>>())))

// Stores of the new state and loads of a row's own state (each touched once per
// step).  When the step's state exceeds the Infinity Cache (`stream`), they are
// non-temporal: caching them would only evict the neighbour rows that the gathers
// of later rows reuse, and the next step cannot find them in cache anyway.
// (A template parameter, not a run-time flag: the compiler merges two otherwise equal
// stores and drops the non-temporal hint.)
template <bool NT, typename VT, typename T>
__device__ __forceinline__ void vstore(T *p, VT v) {
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<VT *>(p));
    else *reinterpret_cast<VT *>(p) = v;
}
template <bool NT, typename VT, typename T>
__device__ __forceinline__ VT vload_own(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const VT *>(p));
    else return *reinterpret_cast<const VT *>(p);
}

// Infinity Cache (memory-side last-level cache) of the MI355X
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;

template <typename T, int RB>
struct VGeo {
    static constexpr int VEC = Vec16<T>::n;
    static constexpr int LPR = RB / VEC;     // lanes per row
    static constexpr int RPW = 64 / LPR;     // rows per wave
    static constexpr int RPB = 4 * RPW;      // rows per 256-thread workgroup (one tile)
    static constexpr int W = 16;             // padded slots per row
};

// LDS image of one tile's row operands.
template <typename T, int RB>
struct TileOps {
    using G = VGeo<T, RB>;
    int col[G::RPB * G::W];
    T kv[G::RPB * G::W];
    T bv[G::RPB * G::W];
    T dm[G::RPB];
    int bo[G::RPB], bn[G::RPB], x0[G::RPB], x1[G::RPB];
};

// Stage the operands of rows [row0, row0 + RPB) (rows >= n get zero weights); the
// B values when need_b (every step of the three-level form needs them).
// Contains __syncthreads(); every thread of the workgroup must call it.
template <typename T, int RB>
__device__ __forceinline__ void stage_tile(const RowOps<T> &o, int n, int row0, bool need_b, TileOps<T, RB> &L) {
    using G = VGeo<T, RB>;
    for (int e = threadIdx.x; e < G::RPB * G::W; e += 256) {
        const int rw = row0 + e / G::W;
        const bool ok = rw < n;
        const int64_t src = int64_t(ok ? rw : 0) * G::W + e % G::W;
        L.col[e] = ok ? o.ecol[src] : 0;
        L.kv[e] = ok ? o.eval[src] : T(0);
    }
    for (int e = threadIdx.x; e < G::RPB; e += 256) {
        const int rw = row0 + e;
        const bool ok = rw < n;
        L.bo[e] = ok ? o.bsoff[rw] : -1;
        L.bn[e] = ok ? o.bnum[rw] : 0;
        L.x0[e] = ok ? o.xptr[rw] : 0;
        L.x1[e] = ok ? o.xptr[rw + 1] : 0;
        L.dm[e] = ok ? o.dtm[rw] : T(0);
    }
    __syncthreads();
    if (need_b) {
        for (int e = threadIdx.x; e < G::RPB * G::W; e += 256) {
            const int bo = L.bo[e / G::W];
            L.bv[e] = bo >= 0 ? o.bslot[bo + e % G::W] : T(0);
        }
        __syncthreads();
    }
}

template <typename VT, typename T>
__device__ __forceinline__ VT vfma(T w, VT x, VT acc) {
    VT o;
#pragma unroll
    for (int i = 0; i < Vec16<T>::n; ++i) o[i] = mad(w, x[i], acc[i]);
    return o;
}

// acc += sum_slots K(row, slot) X[col][q-th vector]; with_b: bacc += B(row, slot)
// bdiff(X[col], Y[col]).  The B sums (boundary rows only) run after the K sums have
// been consumed, with their own gathers, so the two sets of gathers are never live
// together and the kernel keeps the register budget (and occupancy) of the interior
// rows.  Slot 0 of every row is its diagonal, so the first gather is the row's own
// X value; it is returned in `own`.
template <typename T, int RB>
__device__ __forceinline__ void vrow_sums(const RowOps<T> &o, const TileOps<T, RB> &L, int lr, int q,
                                          const T *__restrict__ X, const T *__restrict__ Y, bool with_b,
                                          bool only_prev, typename Vec16<T>::t &acc, typename Vec16<T>::t &bacc,
                                          typename Vec16<T>::t &own) {
    using G = VGeo<T, RB>;
    using VT = typename Vec16<T>::t;
    const int base = lr * G::W;
    constexpr int CH = kGatherChunk;
    // 32-bit byte offsets from the uniform bases (state arrays are < 4 GiB)
    const char *Xc = reinterpret_cast<const char *>(X);
    const char *Yc = reinterpret_cast<const char *>(Y);
    const uint32_t qoff = uint32_t(q) * 16u;
    constexpr uint32_t ROWB = uint32_t(RB * sizeof(T));
#pragma unroll
    for (int j0 = 0; j0 < G::W; j0 += CH) {
        VT x[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j)
            x[j] = *reinterpret_cast<const VT *>(Xc + (uint32_t(L.col[base + j0 + j]) * ROWB + qoff));
        if (j0 == 0) own = x[0];
#pragma unroll
        for (int j = 0; j < CH; ++j) acc = vfma(L.kv[base + j0 + j], x[j], acc);
    }
    const int x0 = L.x0[lr], x1 = L.x1[lr];
    for (int k = x0; k < x1; ++k) {
        const VT xv = *reinterpret_cast<const VT *>(Xc + (uint32_t(o.xcol[k]) * ROWB + qoff));
        acc = vfma(o.xval[k], xv, acc);
    }
    if (with_b) {
        // only the row's first bnum slots carry B; re-read the slot operands from LDS
        // instead of keeping them live across the K sums
        int bbase = base;
        asm volatile("" : "+v"(bbase));
        const int nb = L.bn[lr];
        constexpr int BCH = CH / 4;  // two gathers per slot
#pragma unroll
        for (int j0 = 0; j0 < G::W; j0 += BCH) {
            if (j0 < nb) {
                VT y[BCH];
#pragma unroll
                for (int j = 0; j < BCH; ++j) {
                    y[j] = VT{};
                    if (j0 + j < nb) {
                        const uint32_t off = uint32_t(L.col[bbase + j0 + j]) * ROWB + qoff;
                        const VT xv = *reinterpret_cast<const VT *>(Xc + off);
                        const VT yv = *reinterpret_cast<const VT *>(Yc + off);
#pragma unroll
                        for (int i = 0; i < G::VEC; ++i) y[j][i] = bdiff(xv[i], yv[i], only_prev);
                    }
                }
#pragma unroll
                for (int j = 0; j < BCH; ++j) bacc = vfma(L.bv[bbase + j0 + j], y[j], bacc);
            }
        }
        for (int k = x0; k < x0 + nb - G::W; ++k) {
            const uint32_t off = uint32_t(o.xcol[k]) * ROWB + qoff;
            const VT xv = *reinterpret_cast<const VT *>(Xc + off);
            const VT yv = *reinterpret_cast<const VT *>(Yc + off);
            VT dv;
#pragma unroll
            for (int i = 0; i < G::VEC; ++i) dv[i] = bdiff(xv[i], yv[i], only_prev);
            bacc = vfma(o.bslot[L.bo[lr] + G::W + (k - x0)], dv, bacc);
        }
    }
}

template <typename T>
struct VFwdArgs {
    RowOps<T> o;
    const int32_t *snode;
    const T *sw;
    const T *S, *Sp;  // S^n, S^{n-1}
    T *Sn;            // S^{n+1}
    void *y;
    double yscale;
    int n, n_obs, n_tiles, n_samp, sample, t;
    int stream;  // state beyond the Infinity Cache: launch the non-temporal variant
    T dt;
    // halo tiles (HaloTiles), float32 blocks of 256-byte row chunks
    const int32_t *hdesc, *hrow;
    const uint32_t *hmeta;
    int n_ht;
};

// Sampling block j of a forward step: y = Pi (S^n + S^{n-1})/2 of the incoming
// state, one lane per (sensor, rhs).
template <typename T, typename OT, int RB>
__device__ __forceinline__ void fwd_sample(const VFwdArgs<T> &a, int j) {
    const int64_t e = int64_t(j) * 256 + threadIdx.x;
    if (e >= int64_t(a.n_obs) * RB) return;
    const int s = int(e / RB), r = int(e % RB);
    T y = T(0);
    for (int k = 0; k < 4; ++k) {
        const int64_t id = int64_t(a.snode[4 * s + k]) * RB + r;
        y = mad(a.sw[4 * s + k], T(0.5) * (a.S[id] + a.Sp[id]), y);
    }
    OT *yo = static_cast<OT *>(a.y);
    yo[(int64_t(a.t) * a.n_obs + s) * RB + r] = static_cast<OT>(static_cast<double>(y) * a.yscale);
}

// Forward step (same update as k_fwd) with vector lanes on logical tile `tile`;
// the tiles after the row tiles write the samples of the incoming state.
template <typename T, typename OT, int RB, bool NT>
__device__ __forceinline__ void fwd_tile(const VFwdArgs<T> &a, int tile, TileOps<T, RB> &L) {
    using G = VGeo<T, RB>;
    using VT = typename Vec16<T>::t;
    if (tile < a.n_tiles) {
        const int row0 = tile * G::RPB;
        stage_tile<T, RB>(a.o, a.n, row0, true, L);
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int lr = wave * G::RPW + lane / G::LPR, q = lane % G::LPR;
        const int row = row0 + lr;
        if (row < a.n) {
            const int64_t id = int64_t(row) * RB + q * G::VEC;
            VT acc = {}, bacc = {}, cur;
            vrow_sums<T, RB>(a.o, L, lr, q, a.S, a.Sp, L.bo[lr] >= 0, false, acc, bacc, cur);
            // loaded after the sums: the kernel has no register to spare for it before
            const VT prev = vload_own<NT, VT>(a.Sp + id);
            const T dm = L.dm[lr];
            VT sn;
#pragma unroll
            for (int i = 0; i < G::VEC; ++i) sn[i] = step_update(cur[i], prev[i], acc[i], bacc[i], T(0), dm, a.dt);
            vstore<NT, VT>(a.Sn + id, sn);
        }
    } else if (a.sample) {
        fwd_sample<T, OT, RB>(a, tile - a.n_tiles);
    }
}

template <typename T, typename OT, int RB, bool NT>
__global__ void __launch_bounds__(256) PAT_VOCC(T, RB) k_fwd_v(const VFwdArgs<T> a) {
    __shared__ TileOps<T, RB> L;
    fwd_tile<T, OT, RB, NT>(a, fwd_work(xcd_tile(blockIdx.x, gridDim.x), a.n_tiles, a.n_samp), L);
}

// Several meshes in one launch; mesh m has tiles[m] logical tiles.  Every XCD
// takes one eighth of each mesh (a contiguous range of its k-d order), as a
// launch of that mesh alone would, so each mesh's state stays spread over all
// eight L2 caches: XCD x walks, mesh after mesh, tiles
// [x q_m + min(x, r_m), +q_m + (x < r_m)) with q_m = tiles[m] / 8, r_m = tiles[m] % 8.
// The grid is 8 x the largest per-XCD count; blocks past their XCD's count idle.
template <typename A>
struct Multi {
    A a[kMaxMeshes];
    int tiles[kMaxMeshes];
    int n;
};

template <typename T, typename OT, int RB, bool NT>
__global__ void __launch_bounds__(256) PAT_VOCC(T, RB) k_fwd_vm(const Multi<VFwdArgs<T>> mm) {
    __shared__ TileOps<T, RB> L;
    int m, local;
    if (!mesh_tile(mm.tiles, mm.n, blockIdx.x, &m, &local, false)) return;
    fwd_tile<T, OT, RB, NT>(mm.a[m], fwd_work(local, mm.a[m].n_tiles, mm.a[m].n_samp), L);
}

template <typename T>
struct VAdjArgs {
    RowOps<T> o;
    const int32_t *injptr, *injs;
    const T *injw;
    const T *S, *Sp;  // q_k, q_{k-1}
    T *Sn;            // q_{k+1}, or the result after the last step
    const void *yh;
    double yscale;
    int n, n_obs, n_tiles, last;
    int ta, tb;  // sources: Pi^T yhat at sample indices ta (if >= 0) and tb
    int stream;  // state beyond the Infinity Cache: launch the non-temporal variant
    T dt;
    const int32_t *hdesc, *hrow;
    const uint32_t *hmeta;
    int n_ht;
};

// Pi^T (yhat^{ta} + yhat^{tb}) over the injection entries [e0, e1) of a row, for
// the VEC right-hand sides from rhs0 (yhat^{ta} left out for ta < 0).
template <typename T, typename YT, int RB, typename VT>
__device__ __forceinline__ VT vinject(const VAdjArgs<T> &a, int e0, int e1, int rhs0) {
    VT inj = {};
    const YT *yh = static_cast<const YT *>(a.yh);
    for (int e = e0; e < e1; ++e) {
        const int s = a.injs[e];
        const int64_t sb = (int64_t(a.tb) * a.n_obs + s) * RB + rhs0;
        const int64_t sa = (int64_t(a.ta) * a.n_obs + s) * RB + rhs0;
        const T w = a.injw[e];
#pragma unroll
        for (int i = 0; i < Vec16<T>::n; ++i) {
            T v = static_cast<T>(static_cast<double>(yh[sb + i]) * a.yscale);
            if (a.ta >= 0) v = static_cast<T>(static_cast<double>(yh[sa + i]) * a.yscale) + v;
            inj[i] = mad(w, v, inj[i]);
        }
    }
    return inj;
}

// Transposed step (same update as k_adj) with vector lanes on logical tile `tile`.
template <typename T, typename YT, int RB, bool NT>
__device__ __forceinline__ void adj_tile(const VAdjArgs<T> &a, int tile, TileOps<T, RB> &L) {
    using G = VGeo<T, RB>;
    using VT = typename Vec16<T>::t;
    if (tile >= a.n_tiles) return;
    const int row0 = tile * G::RPB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool winj = wave_injects(a.injptr, row0 + wave * G::RPW, G::RPW, a.n);
    stage_tile<T, RB>(a.o, a.n, row0, true, L);
    const int lr = wave * G::RPW + lane / G::LPR, q = lane % G::LPR;
    const int row = row0 + lr;
    if (row >= a.n) return;
    const int64_t id = int64_t(row) * RB + q * G::VEC;
    VT kq = {}, bq = {}, cur;
    vrow_sums<T, RB>(a.o, L, lr, q, a.S, a.Sp, L.bo[lr] >= 0, a.last, kq, bq, cur);
    // loaded after the sums: the kernel has no register to spare for it before
    const VT prev = vload_own<NT, VT>(a.Sp + id);
    const T dm = L.dm[lr];
    VT inj = {};
    if (winj) inj = vinject<T, YT, RB, VT>(a, a.injptr[row], a.injptr[row + 1], q * G::VEC);
    VT out;
#pragma unroll
    for (int i = 0; i < G::VEC; ++i) {
        const T src = T(0.5) * inj[i];
        out[i] = a.last ? adj_result(cur[i], prev[i], kq[i], bq[i], src, dm, a.dt)
                        : step_update(cur[i], prev[i], kq[i], bq[i], src, dm, a.dt);
    }
    vstore<NT, VT>(a.Sn + id, out);
}

template <typename T, typename YT, int RB, bool NT>
__global__ void __launch_bounds__(256) PAT_VOCC(T, RB) k_adj_v(const VAdjArgs<T> a) {
    __shared__ TileOps<T, RB> L;
    adj_tile<T, YT, RB, NT>(a, xcd_tile_rev(blockIdx.x, gridDim.x), L);
}

template <typename T, typename YT, int RB, bool NT>
__global__ void __launch_bounds__(256) PAT_VOCC(T, RB) k_adj_vm(const Multi<VAdjArgs<T>> mm) {
    __shared__ TileOps<T, RB> L;
    int m, local;
    if (!mesh_tile(mm.tiles, mm.n, blockIdx.x, &m, &local, true)) return;
    adj_tile<T, YT, RB, NT>(mm.a[m], local, L);
}

// ---------------------------------------------------------------------------
// Halo step kernels: float32 blocks whose rows are 64, 128 or 256 RHS (one to
// four 256-byte chunks).
//
// The vector-lane kernels above gather 16 neighbour rows per row through the
// CU's texture units, which keeps those units busy most of the step.  Here a
// tile of consecutive rows (HaloTiles: at most 32 rows whose distinct neighbour
// rows, the halo, fit 132 LDS rows; on the 195,112-node ball 4.7 halo rows per
// row) copies its halo and its row operands from memory straight into LDS
// (global_load_lds_dwordx4, 64 lanes x 16 bytes per instruction, no registers
// in between), and every slot reads its neighbour from there.  Each workgroup
// (512 threads: 32 rows x 16 lanes of 16 bytes) walks its tiles in a loop with
// two LDS buffers: while it computes one tile, the copies of the next are in
// flight, and the stores of the previous one drain.  Work item = (row chunk,
// tile); XCD x takes the x-th eighth of the tiles, its workgroups interleaved
// over them, so the tiles in flight on one XCD are neighbours and share their
// halo rows in that XCD's L2.  The halo holds rows of the state S (the K part)
// and, at the rows that its boundary slots refer to, rows of the previous state
// S_prev (the B part).  Each lane of a
// row's 16 reads one slot's operands from the LDS image and hands them to the
// others by DPP row broadcast.  Sums run in the slot order of the vector-lane
// kernels, with the same operations, so both give the same bits.
// ---------------------------------------------------------------------------

using F4 = Vec16<float>::t;  // 16 bytes of float32
constexpr int kHRows = HaloTiles::kRows;
constexpr int kHMax = HaloTiles::kMax;
constexpr int kHMetaWords = HaloTiles::kMetaBytes / 4;
constexpr int kHThreads = kHRows * 16;
constexpr int kHWaves = kHThreads / 64;
constexpr int kHPerWave = (kHMax / 4 + kHWaves - 1) / kHWaves;  // halo copy instructions per wave at most
constexpr int kHChunk = 4;  // LDS reads in flight per lane before they are consumed
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
static_assert(kHThreads % 64 == 0 && kHThreads <= 1024 && (kHMetaWords + 255) / 256 <= kHWaves, "halo tile geometry");

// LDS image of one tile
struct alignas(16) HaloBuf {
    F4 rows[kHMax * 16];      // halo rows (256-byte chunks): K part, then B part
    uint32_t meta[kHMetaWords];   // the tile's metadata block (HaloTiles)
};
// LDS of a workgroup: two tile images and two halo row lists, each its own
// __shared__ variable, so that the compiler can tell the copies into one buffer
// from the reads of the other and does not wait for the former before the latter
struct alignas(16) HaloList {  // copied into 16 bytes per lane
    int32_t r[kHMax];
};
// workgroups per CU that the LDS of two tile images and two lists allows (160 KiB per CU)
constexpr int kHPerCU = int(163840 / (2 * (sizeof(HaloBuf) + sizeof(HaloList))));
static_assert(kHPerCU >= 1, "one workgroup per CU at least");

struct HDesc {
    int r0, nr, h0, nk4, nb4, moff, mbytes, nbr;
};

// unpack a tile descriptor (HaloTiles::desc) into wave-uniform values
__device__ __forceinline__ HDesc desc_uniform(const int4 u) {
    const int r0 = __builtin_amdgcn_readfirstlane(u.x), h0 = __builtin_amdgcn_readfirstlane(u.y);
    const int moff = __builtin_amdgcn_readfirstlane(u.z), f = __builtin_amdgcn_readfirstlane(u.w);
    constexpr int B = HaloTiles::kNrBits, M = (1 << B) - 1;
    const int nr = f & M, nk4 = (f >> B) & 255, nb4 = (f >> (B + 8)) & 255, nbr = (f >> (B + 16)) & M;
    return {r0, nr, h0, nk4, nb4, moff, nr * 96 + nbr * 80, nbr};
}

// Work items of this workgroup: (chunk c, tile t).  XCD x (workgroups b with
// b % 8 == x) owns the x-th eighth of the tiles, [t_lo, t_lo + ntx), seen as rows
// of G8 consecutive tiles (one per workgroup of the XCD: neighbouring tiles are in
// flight together and share halo rows in its L2).  Two workgroups share a CU, and
// the one dispatched first (k = b / 8 < G8 / 2) runs about a fifth faster than
// the other; so every kRowPeriod-th row goes to the first half only, two tiles
// each, and they take 10 tiles for every 8 of the others.  A workgroup walks its
// tiles in row order, once per 256-byte chunk.
struct HWork {
    int t_lo, ntx, k, G8, per_c, n;
    bool weighted, first_half;
    // local index (tile - t_lo) of this workgroup's j-th tile; increasing in j
    __device__ int local(int j) const { return hwork_local(j, G8, k, weighted, first_half); }
    __device__ HWork(int n_ht, int NC) {
        G8 = int(gridDim.x >> 3);
        const int x = int(blockIdx.x & 7);
        k = int(blockIdx.x >> 3);
        t_lo = int(int64_t(n_ht) * x / 8);
        ntx = int(int64_t(n_ht) * (x + 1) / 8) - t_lo;
        weighted = kHPerCU == 2 && G8 % 2 == 0;
        first_half = 2 * k < G8;
        per_c = 0;
        while (local(per_c) < ntx) ++per_c;
        n = per_c * NC;
    }
    __device__ int chunk(int it) const { return it / per_c; }
    __device__ int tile(int it) const { return t_lo + local(it - chunk(it) * per_c); }
};

__device__ __forceinline__ void lds_copy16(const void *src, void *lds) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

// Start the copy of a tile's halo row list (nh entries, a multiple of 4 from a
// 16-byte aligned start) into list; one wave issues it.
__device__ __forceinline__ void halo_list_issue(const int32_t *hrow, const HDesc &d, int nh, int32_t *list, int wave,
                                                int lane) {
    if (wave == 1 && 4 * lane < nh) lds_copy16(hrow + d.h0 + 4 * lane, list);
}

// Start the copies of a tile into Lb: its nh halo rows (row numbers from list; the
// first nk4 from X, the rest from Y) at byte offset coff of each row, and its
// metadata block.  Copy instruction h (halo rows 4h .. 4h+3) is issued by wave h % 8.
template <uint32_t RS>
__device__ __forceinline__ void halo_issue(const char *X, const char *Y, uint32_t coff, const uint32_t *hmeta,
                                           const HDesc &d, int nh, const int32_t *list, HaloBuf &Lb, int wave,
                                           int lane) {
    // wave is wave-uniform (callers pass it through readfirstlane), so the tests and
    // the base select below are scalar; the list entries are read in one batch
    int hr[kHPerWave];
#pragma unroll
    for (int m = 0; m < kHPerWave; ++m) {
        const int h = wave + kHWaves * m;
        hr[m] = list[min(4 * h, kHMax - 4) + (lane >> 4)];
    }
    const uint32_t lo = coff + uint32_t(lane & 15) * 16u;
#pragma unroll
    for (int m = 0; m < kHPerWave; ++m) {
        const int h = wave + kHWaves * m;
        if (4 * h < nh) {
            const char *base = 4 * h < d.nk4 ? X : Y;
            lds_copy16(base + (uint32_t(hr[m]) * RS + lo), &Lb.rows[h * 64]);
        }
    }
    const int nu = d.mbytes >> 4, u = kHWaves - 1 - wave;  // metadata: 16-byte units, 64 per instruction
    if (u * 64 < nu && u * 64 + lane < nu)
        lds_copy16(hmeta + 4 * (int64_t(d.moff) + u * 64 + lane), &Lb.meta[u * 256]);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = B, B + S, ... < E.
template <int B, int E, int S = 1, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + S, E, S>(f);
    }
}

// Lane J of this lane's row of 16 lanes (DPP row broadcast): the 16 lanes of a row
// group each hold one slot's operands and hand them to the group slot by slot.
template <int J>
__device__ __forceinline__ uint32_t row_bcast(uint32_t x) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x150 + J, 0xF, 0xF, true));
}
template <int J>
__device__ __forceinline__ float row_bcast(float x) {
    return __uint_as_float(row_bcast<J>(__float_as_uint(x)));
}

// The operands of row g of the tile in Lb (metadata layout of HaloTiles) as held by
// lane q of its row group: slot q's K value and K-halo byte offset, and info word
// q % 4.  Per-row values come from the info words by row broadcast.
struct HLane {
    uint32_t koff;  // byte offset of slot q's neighbour in the K part of the halo
    float kv;
    uint32_t info;
};
__device__ __forceinline__ HLane halo_lane(const HaloBuf &Lb, int nr, int g, int q) {
    HLane h;
    h.koff = uint32_t(reinterpret_cast<const uint8_t *>(Lb.meta + g * 4)[q]) * 256u;
    h.info = Lb.meta[nr * 4 + g * 4 + (q & 3)];
    h.kv = reinterpret_cast<const float *>(Lb.meta + nr * 8 + g * 16)[q];
    return h;
}
// per-row values from the info words: dt/m, boundary row (0xFF: none), bnum, the
// overflow range [x0, x0 + nx) and the injection range [inj0, inj0 + ninj)
__device__ __forceinline__ float hl_dm(const HLane &h) { return __uint_as_float(row_bcast<0>(h.info)); }
__device__ __forceinline__ uint32_t hl_word(const HLane &h) { return row_bcast<1>(h.info); }
__device__ __forceinline__ int hl_x0(const HLane &h) { return int(row_bcast<2>(h.info)); }
__device__ __forceinline__ int hl_inj0(const HLane &h) { return int(row_bcast<3>(h.info)); }
__device__ __forceinline__ int hw_brow(uint32_t w) { return int(w & 0xFFu); }
__device__ __forceinline__ int hw_bnum(uint32_t w) { return int((w >> 8) & 0xFFu); }
__device__ __forceinline__ int hw_nx(uint32_t w) { return int((w >> 16) & 0xFFu); }
__device__ __forceinline__ int hw_ninj(uint32_t w) { return int(w >> 24); }
// boundary row br's B value and B-halo byte offset (base: the B part's first row) of slot q
__device__ __forceinline__ float hb_value(const HaloBuf &Lb, int nr, int br, int q) {
    return reinterpret_cast<const float *>(Lb.meta + nr * 24 + br * 16)[q];
}
__device__ __forceinline__ uint32_t hb_offset(const HaloBuf &Lb, int nr, int nbr, int br, int q, int base) {
    return (uint32_t(base) + reinterpret_cast<const uint8_t *>(Lb.meta + nr * 24 + nbr * 16 + br * 4)[q]) * 256u;
}

__device__ __forceinline__ F4 lds_row(const HaloBuf &Lb, uint32_t off) {
    return *reinterpret_cast<const F4 *>(reinterpret_cast<const char *>(Lb.rows) + off);
}

// acc += sum_slots K(row, slot) X[col] from the halo, slot order as vrow_sums, then
// the entries beyond 16 from memory; own = slot 0 (the row's diagonal).
__device__ __forceinline__ void halo_ksums(const HaloBuf &Lb, const HLane &h, uint32_t q16, int x0, int x1,
                                           const float *__restrict__ xval, const int32_t *__restrict__ xcol,
                                           const char *Xc, uint32_t RS, uint32_t coff, F4 &acc, F4 &own) {
    static_for<0, 16, kHChunk>([&](auto J0) {
        constexpr int j0 = decltype(J0)::value;
        F4 x[kHChunk];
        static_for<0, kHChunk>([&](auto J) { x[J.value] = lds_row(Lb, row_bcast<j0 + J.value>(h.koff) + q16); });
        if constexpr (j0 == 0) own = x[0];
        static_for<0, kHChunk>([&](auto J) { acc = vfma(row_bcast<j0 + J.value>(h.kv), x[J.value], acc); });
    });
    for (int k = x0; k < x1; ++k) {
        const F4 xv = *reinterpret_cast<const F4 *>(Xc + (uint32_t(xcol[k]) * RS + coff + q16));
        acc = vfma(xval[k], xv, acc);
    }
}

// bacc += sum over the first nb slots of B(row, slot) bdiff(X[col], Y[col]), as
// vrow_sums: slot j's X row at the halo byte offset koffq of lane j (the K part), its
// Y row at boffq of lane j (the B part), the entries beyond 16 from memory.  bwq:
// this lane's slot's B value.
__device__ __forceinline__ void halo_bsums(const HaloBuf &Lb, uint32_t koffq, uint32_t boffq, float bwq, int nb,
                                           uint32_t q16, const float *__restrict__ bslot, int bo,
                                           const int32_t *__restrict__ xcol, int x0, const char *Xc, const char *Yc,
                                           uint32_t RS, uint32_t coff, bool only_prev, F4 &bacc) {
    // re-read the K part's rows from LDS instead of keeping the K sums' reads live
    asm volatile("" : "+v"(koffq));
    // slots j >= nb carry B = 0: the vector-lane kernels add 0 * 0 there, which leaves
    // bacc unchanged (it starts at +0 and a sum that starts at +0 never becomes -0),
    // so skipping them keeps the bits
    static_for<0, 16, kHChunk>([&](auto J0) {
        constexpr int j0 = decltype(J0)::value;
        if (j0 < nb) {
            F4 y[kHChunk];
            static_for<0, kHChunk>([&](auto J) {
                if (j0 + J.value < nb) {
                    const F4 xv = lds_row(Lb, row_bcast<j0 + J.value>(koffq) + q16);
                    const F4 yv = lds_row(Lb, row_bcast<j0 + J.value>(boffq) + q16);
#pragma unroll
                    for (int i = 0; i < 4; ++i) y[J.value][i] = bdiff(xv[i], yv[i], only_prev);
                }
            });
            static_for<0, kHChunk>([&](auto J) {
                if (j0 + J.value < nb) bacc = vfma(row_bcast<j0 + J.value>(bwq), y[J.value], bacc);
            });
        }
    });
    for (int k = x0; k < x0 + nb - 16; ++k) {
        const uint32_t off = uint32_t(xcol[k]) * RS + coff + q16;
        const F4 xv = *reinterpret_cast<const F4 *>(Xc + off);
        const F4 yv = *reinterpret_cast<const F4 *>(Yc + off);
        F4 dv;
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[i] = bdiff(xv[i], yv[i], only_prev);
        bacc = vfma(bslot[bo + 16 + (k - x0)], dv, bacc);
    }
}

// Pipeline of one workgroup over its work items: fn_list(d, list) starts the copy
// of an item's halo row list, fn_issue(it, d, list, buffer) the copies of its halo
// and metadata, fn_pre(it, d) loads its own rows into the "next" registers and
// fn_rot moves them to the "current" ones, fn_compute(it, d, buffer) computes
// item it into registers and fn_store() writes the last computed item.  While
// item it is computed, the copies of item it + 1, the row list of item it + 2 and
// the descriptor of item it + 4 are in flight, and item it - 1's stores drain.
// Even items use (B0, L0), odd items (B1, L1); the loop is unrolled by two so
// that each access names its buffer at compile time.
template <typename List, typename Issue, typename Pre, typename Rot, typename Compute, typename Store>
__device__ __forceinline__ void halo_loop(const HWork &wk, const int32_t *hdesc, HaloBuf &B0, HaloBuf &B1,
                                          HaloList &L0, HaloList &L1, List fn_list, Issue fn_issue, Pre fn_pre,
                                          Rot fn_rot, Compute fn_compute, Store fn_store) {
    const int n = wk.n;
    if (n == 0) return;
    const int4 *D = reinterpret_cast<const int4 *>(hdesc);
    auto raw = [&](int it) { return it < n ? D[wk.tile(it)] : int4{0, 0, 0, 0}; };
    HDesc d0 = desc_uniform(raw(0)), d1 = desc_uniform(raw(1)), d2 = desc_uniform(raw(2));
    fn_list(d0, L0.r);
    if (1 < n) fn_list(d1, L1.r);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    fn_issue(0, d0, L0.r, B0);
    fn_pre(0, d0);
    int4 u3 = raw(3);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copies of item 0 have landed
    __syncthreads();
    auto step = [&](int it, HaloBuf &Bc, HaloBuf &Bn, HaloList &Lc, HaloList &Ln) {
        fn_rot();
        if (it + 1 < n) fn_issue(it + 1, d1, Ln.r, Bn);
        if (it + 2 < n) fn_list(d2, Lc.r);
        if (it > 0) fn_store();
        if (it + 1 < n) fn_pre(it + 1, d1);
        const int4 u4 = raw(it + 4);
        fn_compute(it, d0, Bc);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copies of item it + 1 and list it + 2 have landed
        __syncthreads();                     // ... for every wave, and item it's buffer is free
        d0 = d1;
        d1 = d2;
        d2 = desc_uniform(u3);
        u3 = u4;
    };
    for (int it = 0; it < n; it += 2) {
        step(it, B0, B1, L0, L1);
        if (it + 1 < n) step(it + 1, B1, B0, L1, L0);
    }
    fn_store();
}

// One halo-tile step (forward: FWD, no sources; transposed: sources, and with LAST the
// closing launch).  The K part of a tile's halo holds rows of S, the B part rows of
// Sp; each row's own Sp comes from memory one item ahead.  (LAST is a template
// parameter: as a run-time flag its selects cost 2% of every step.)
template <bool FWD, bool LAST, int RB, bool NT, typename Args, typename Src>
__device__ __forceinline__ void halo_step(const Args &a, Src fn_src) {
    constexpr int NC = RB / 64;
    constexpr uint32_t RS = uint32_t(RB) * 4u;
    __shared__ HaloBuf B0, B1;
    __shared__ HaloList L0, L1;
    const int tid = int(threadIdx.x), wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, g = tid >> 4,
              q = tid & 15;
    const HWork wk(a.n_ht, NC);
    const char *Sc = reinterpret_cast<const char *>(a.S);
    const char *Spc = reinterpret_cast<const char *>(a.Sp);
    F4 prev_cur = {}, prev_nxt = {}, out = {};
    uint32_t out_id = kNoRow;  // byte offset of the pending result, kNoRow: none
    auto fn_list = [&](const HDesc &d, int32_t *list) {
        halo_list_issue(a.hrow, d, d.nk4 + d.nb4, list, wave, lane);
    };
    auto fn_issue = [&](int it, const HDesc &d, const int32_t *list, HaloBuf &Bn) {
        halo_issue<RS>(Sc, Spc, uint32_t(wk.chunk(it)) * 256u, a.hmeta, d, d.nk4 + d.nb4, list, Bn, wave, lane);
    };
    auto fn_pre = [&](int it, const HDesc &d) {
        if (g < d.nr)
            prev_nxt = vload_own<NT, F4>(reinterpret_cast<const float *>(
                Spc + (uint32_t(d.r0 + g) * RS + uint32_t(wk.chunk(it)) * 256u + uint32_t(q) * 16u)));
    };
    auto fn_rot = [&]() { prev_cur = prev_nxt; };
    auto fn_store = [&]() {
        if (out_id != kNoRow) vstore<NT, F4>(reinterpret_cast<float *>(reinterpret_cast<char *>(a.Sn) + out_id), out);
    };
    auto fn_compute = [&](int it, const HDesc &d, const HaloBuf &Lb) {
        out_id = kNoRow;
        if (g >= d.nr) return;
        const int c = wk.chunk(it);
        const uint32_t coff = uint32_t(c) * 256u, q16 = uint32_t(q) * 16u;
        const HLane h = halo_lane(Lb, d.nr, g, q);
        const uint32_t hw = hl_word(h);
        const int x0 = hl_x0(h), x1 = x0 + hw_nx(hw);
        F4 acc = {}, bacc = {}, cur;
        halo_ksums(Lb, h, q16, x0, x1, a.o.xval, a.o.xcol, Sc, RS, coff, acc, cur);
        const int row = d.r0 + g;
        if (hw_brow(hw) != 0xFF) {
            const int nb = hw_bnum(hw), br = hw_brow(hw);
            const int bo = nb > 16 ? a.o.bsoff[row] : 0;
            halo_bsums(Lb, h.koff, hb_offset(Lb, d.nr, d.nbr, br, q, d.nk4), hb_value(Lb, d.nr, br, q), nb, q16,
                       a.o.bslot, bo, a.o.xcol, x0, Sc, Spc, RS, coff, LAST, bacc);
        }
        const float dm = hl_dm(h);
        F4 inj = {};
        if constexpr (!FWD) {
            const int e0 = hl_inj0(h), e1 = e0 + hw_ninj(hw);
            if (e1 > e0) inj = fn_src(e0, e1, c * 64 + q * 4);
        }
        F4 res;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float src = 0.5f * inj[i];
            if constexpr (LAST) res[i] = adj_result(cur[i], prev_cur[i], acc[i], bacc[i], src, dm, a.dt);
            else res[i] = step_update(cur[i], prev_cur[i], acc[i], bacc[i], src, dm, a.dt);
        }
        out = res;
        out_id = uint32_t(row) * RS + coff + q16;
    };
    halo_loop(wk, a.hdesc, B0, B1, L0, L1, fn_list, fn_issue, fn_pre, fn_rot, fn_compute, fn_store);
}

template <typename OT, int RB, bool NT>
__global__ void __launch_bounds__(kHThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_fwd_h(const VFwdArgs<float> a) {
    halo_step<true, false, RB, NT>(a, [](int, int, int) { return F4{}; });
    if (a.sample) {
        // y = Pi (S^n + S^{n-1})/2 of the incoming state, one lane per (sensor, rhs)
        const int64_t total = int64_t(a.n_obs) * RB;
        OT *yo = static_cast<OT *>(a.y);
        for (int64_t e = int64_t(blockIdx.x) * kHThreads + threadIdx.x; e < total;
             e += int64_t(gridDim.x) * kHThreads) {
            const int s = int(e / RB), rr = int(e % RB);
            float y = 0.0f;
            for (int k = 0; k < 4; ++k) {
                const int64_t id = int64_t(a.snode[4 * s + k]) * RB + rr;
                y = mad(a.sw[4 * s + k], 0.5f * (a.S[id] + a.Sp[id]), y);
            }
            yo[(int64_t(a.t) * a.n_obs + s) * RB + rr] = static_cast<OT>(static_cast<double>(y) * a.yscale);
        }
    }
}

template <typename YT, int RB, bool NT, bool LAST>
__global__ void __launch_bounds__(kHThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_adj_h(const VAdjArgs<float> a) {
    halo_step<false, LAST, RB, NT>(a, [&](int e0, int e1, int rhs0) { return vinject<float, YT, RB, F4>(a, e0, e1, rhs0); });
}

// q_{-1} = 0 and q_0 = (dt/2m) Pi^T yhat^{tb} (tb = N_T - 1, the last sample)
template <typename T, typename YT, int RB>
__global__ void __launch_bounds__(256) k_adj_init(const AdjArgs<T> a, T *q0, T *qm1) {
    const int64_t total = int64_t(a.n) * RB;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int row = int(e / RB), r = int(e % RB);
        q0[e] = T(0.5) * a.o.dtm[row] * inject<T, YT, RB>(a, row, r);
        qm1[e] = T(0);
    }
}

// ---------------------------------------------------------------------------
// Layout conversions (LDS-tiled transposes)
// ---------------------------------------------------------------------------

// out[c][r] = in[rb0 + r][perm(c)] (zero for rb0 + r >= R), tile of 64 columns x 64 RHS,
// the block's RHS in chunks of 64
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_pack(const TI *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                                              const int32_t *perm, TO *out) {
    __shared__ double tile[64][65];
    const int64_t c0 = int64_t(blockIdx.x) * 64;
    for (int r0 = 0; r0 < RB; r0 += 64) {
        const int rn = RB - r0 < 64 ? RB - r0 : 64;
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int r = e / 64, c = e % 64;
            const int64_t cc = c0 + c, rr = rb0 + r0 + r;
            double v = 0.0;
            if (cc < cols && rr < R) v = static_cast<double>(in[rr * cols + (perm ? perm[cc] : cc)]);
            tile[r][c] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int c = e / rn, r = e % rn;
            const int64_t cc = c0 + c;
            if (cc < cols) out[cc * RB + r0 + r] = static_cast<TO>(tile[r][c]);
        }
        __syncthreads();
    }
}

// out[rb0 + r][perm(c)] = in[c][r] for rb0 + r < R (same tiling as k_pack)
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_unpack(const TI *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                                                const int32_t *perm, TO *out) {
    __shared__ double tile[64][65];
    const int64_t c0 = int64_t(blockIdx.x) * 64;
    for (int r0 = 0; r0 < RB; r0 += 64) {
        const int rn = RB - r0 < 64 ? RB - r0 : 64;
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int c = e / rn, r = e % rn;
            const int64_t cc = c0 + c;
            tile[r][c] = cc < cols ? static_cast<double>(in[cc * RB + r0 + r]) : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int r = e / 64, c = e % 64;
            const int64_t cc = c0 + c, rr = rb0 + r0 + r;
            if (cc < cols && rr < R) out[rr * cols + (perm ? perm[cc] : cc)] = static_cast<TO>(tile[r][c]);
        }
        __syncthreads();
    }
}

// ---- counter-based standard normals -------------------------------------
// Philox4x64-10 (Salmon et al., SC'11) and the Box-Muller transform.  Normal j
// of stream (seed, kind, k) is lane j%4 of the cipher block with counter
// (j/4, k, kind, 0) and key (seed, 0); lanes (0,1) and (2,3) are Box-Muller
// pairs with u1 = 1 - U(w_even) in (0, 1], u2 = U(w_odd), U(w) = (w >> 11) 2^-53.
struct Normals4 {
    double z[4];
};

__device__ inline Normals4 philox_normals(uint64_t seed, uint64_t kind, uint64_t k, uint64_t blk) {
    uint64_t c0 = blk, c1 = k, c2 = kind, c3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ULL, c0), lo0 = 0xD2E7470EE14C6C93ULL * c0;
        const uint64_t hi1 = __umul64hi(0xCA5A826395121157ULL, c2), lo1 = 0xCA5A826395121157ULL * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    Normals4 o;
    const uint64_t w[4] = {c0, c1, c2, c3};
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        const double u1 = 1.0 - double(w[2 * pr] >> 11) * 0x1p-53;
        const double u2 = double(w[2 * pr + 1] >> 11) * 0x1p-53;
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586476925286766559 * u2;
        o.z[2 * pr] = rad * cos(ang);
        o.z[2 * pr + 1] = rad * sin(ang);
    }
    return o;
}

// out[s*len + j] = normal j of stream (seed, kind, k0 + s)
__global__ void __launch_bounds__(256) k_normals(uint64_t seed, int kind, int64_t k0, int64_t S, int64_t len,
                                                 double *out) {
    const int64_t nblk = (len + 3) / 4, total = S * nblk;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t sm = e / nblk, b = e % nblk;
        const Normals4 z = philox_normals(seed, uint64_t(kind), uint64_t(k0 + sm), uint64_t(b));
#pragma unroll
        for (int l = 0; l < 4; ++l)
            if (4 * b + l < len) out[sm * len + 4 * b + l] = z.z[l];
    }
}

// bd[m][r] = yobs[m] * isig + eta_{k0+rb0+r}[m] drawn on the fly (zero rows past S)
__global__ void __launch_bounds__(256) k_build_rhs_rng(const double *yobs, uint64_t seed, int64_t k0, int64_t S,
                                                       int64_t rb0, int RB, int64_t M, double isig, double *bd) {
    const int64_t nblk = (M + 3) / 4, total = nblk * RB;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = e / RB;
        const int r = int(e % RB);
        const bool live = rb0 + r < S;
        Normals4 z{};
        if (live) z = philox_normals(seed, 0, uint64_t(k0 + rb0 + r), uint64_t(b));
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int64_t m = 4 * b + l;
            if (m < M) bd[m * RB + r] = live ? yobs[m] * isig + z.z[l] : 0.0;
        }
    }
}

// xi[q][r] = normal perm(q) of stream (seed, 1, k0+rb0+r), internal node order (zero rows past S)
__global__ void __launch_bounds__(256) k_xi_rng(uint64_t seed, int64_t k0, int64_t S, int64_t rb0, int RB, int64_t N,
                                                const int32_t *perm, double *xi) {
    const int64_t total = N * RB;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t q = e / RB;
        const int r = int(e % RB);
        double v = 0.0;
        if (rb0 + r < S) {
            const int64_t j = perm ? perm[q] : q;
            v = philox_normals(seed, 1, uint64_t(k0 + rb0 + r), uint64_t(j / 4)).z[j % 4];
        }
        xi[e] = v;
    }
}

// bd[m][r] = yobs[m] * isig + eta[rb0 + r][m]  (zero rows past S); RHS in chunks of 64
__global__ void __launch_bounds__(256) k_build_rhs(const double *yobs, const double *eta, int64_t S, int64_t rb0,
                                                   int RB, int64_t M, double isig, double *bd) {
    __shared__ double tile[64][65];
    const int64_t c0 = int64_t(blockIdx.x) * 64;
    for (int r0 = 0; r0 < RB; r0 += 64) {
        const int rn = RB - r0 < 64 ? RB - r0 : 64;
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int r = e / 64, c = e % 64;
            const int64_t cc = c0 + c, rr = rb0 + r0 + r;
            tile[r][c] = (cc < M && rr < S) ? eta[rr * M + cc] : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * rn; e += 256) {
            const int c = e / rn, r = e % rn;
            const int64_t cc = c0 + c;
            if (cc < M) bd[cc * RB + r0 + r] = (rb0 + r0 + r < S) ? yobs[cc] * isig + tile[r][c] : 0.0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// CGLS helpers (float64)
// ---------------------------------------------------------------------------

__global__ void k_fill(double *x, int64_t n, double v) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) x[e] = v;
}

template <typename T>
__global__ void k_cast(const double *x, T *y, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
        y[e] = static_cast<T>(x[e]);
}

// y = L x = M_L^{1/2} x + a M_L^{-1/2} (K1 x)
// float64 value of lane l of v (l wave-uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b), l));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// sum over the entries k of row i of the K1 pattern, in ascending order, of
// fma(K1[k], f_j x[j RB + r], acc) with j = col[k] and f_j = isqrtm[j] (SCALE) or
// the plain x value, for a wave-uniform row i (RB >= 64, one row per wave): lane l
// holds entry k0 + l's column, value and scale, read back by readlane, and the
// gathers go in groups of 16, all issued before the first is used (the same sums
// as entry by entry, in the same order, with a few dependent round trips per row
// instead of one per entry)
template <bool SCALE>
__device__ __forceinline__ double k1_row_wave(const int32_t *rowptr, const int32_t *col, const double *k1,
                                             const double *isqrtm, int i, int RB, int r, const double *x) {
    constexpr int G = 16;
    const int lane = int(threadIdx.x) & 63;
    const int k0 = rowptr[i], ke = rowptr[i + 1];
    double acc = 0.0;
    for (int kb = k0; kb < ke; kb += 64) {
        const int nk = min(64, ke - kb);
        int cl = 0;
        double wl = 0.0, sl = 1.0;
        if (lane < nk) {
            cl = col[kb + lane];
            wl = k1[kb + lane];
            if (SCALE) sl = isqrtm[cl];
        }
        for (int g = 0; g < nk; g += G) {
            double xv[G];
#pragma unroll
            for (int j = 0; j < G; ++j)  // past the end: the last entry again, loaded but not summed
                xv[j] = x[int64_t(__builtin_amdgcn_readlane(cl, min(g + j, nk - 1))) * RB + r];
#pragma unroll
            for (int j = 0; j < G; ++j)
                if (g + j < nk) {
                    const double w = readlane_f64(wl, g + j);
                    acc = SCALE ? __builtin_fma(w, readlane_f64(sl, g + j) * xv[j], acc) : __builtin_fma(w, xv[j], acc);
                }
        }
    }
    return acc;
}

__global__ void __launch_bounds__(256) k_prior(const int32_t *rowptr, const int32_t *col, const double *k1,
                                               const double *sqrtm, const double *isqrtm, int n, int RB, double a,
                                               const double *x, double *y) {
    // 256 / RB rows per block and pass, thread (row lr, RHS r); with RB >= 64 a wave
    // holds one row, whose operands are then wave-uniform (scalar loads)
    const int rpb = 256 / RB, r = int(threadIdx.x) % RB, lr = int(threadIdx.x) / RB;
    auto row = [&](int i, bool wave_row) {
        double acc = 0.0;
        if (wave_row) {
            acc = k1_row_wave<false>(rowptr, col, k1, isqrtm, i, RB, r, x);
        } else {
#pragma unroll 4
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc = __builtin_fma(k1[k], x[int64_t(col[k]) * RB + r], acc);
        }
        const int64_t e = int64_t(i) * RB + r;
        y[e] = sqrtm[i] * x[e] + a * isqrtm[i] * acc;
    };
    for (int64_t i = int64_t(blockIdx.x) * rpb + lr; i < n; i += int64_t(gridDim.x) * rpb) {
        if (RB >= 64) row(__builtin_amdgcn_readfirstlane(int(i)), true);
        else row(int(i), false);
    }
}

// out = isig * PH + L^T rp,  L^T rp = M_L^{1/2} rp + a K1 (M_L^{-1/2} rp); PH is the
// transpose sweep's result G^T r_d
template <typename T>
__global__ void __launch_bounds__(256) k_gext_t(const int32_t *rowptr, const int32_t *col, const double *k1,
                                                const double *sqrtm, const double *isqrtm, int n, int RB, double a,
                                                double isig, const T *PH, const double *rp, double *out) {
    // as k_prior: 256 / RB rows per block and pass; wave-uniform rows for RB >= 64
    const int rpb = 256 / RB, r = int(threadIdx.x) % RB, lr = int(threadIdx.x) / RB;
    auto row = [&](int i, bool wave_row) {
        double acc = 0.0;
        if (wave_row) {
            acc = k1_row_wave<true>(rowptr, col, k1, isqrtm, i, RB, r, rp);
        } else {
#pragma unroll 4
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int j = col[k];
                acc = __builtin_fma(k1[k], isqrtm[j] * rp[int64_t(j) * RB + r], acc);
            }
        }
        const int64_t e = int64_t(i) * RB + r;
        out[e] = isig * static_cast<double>(PH[e]) + (sqrtm[i] * rp[e] + a * acc);
    };
    for (int64_t i = int64_t(blockIdx.x) * rpb + lr; i < n; i += int64_t(gridDim.x) * rpb) {
        if (RB >= 64) row(__builtin_amdgcn_readfirstlane(int(i)), true);
        else row(int(i), false);
    }
}

// y = L^T x = M_L^{1/2} x + a K1 (M_L^{-1/2} x)
__global__ void __launch_bounds__(256) k_prior_t(const int32_t *rowptr, const int32_t *col, const double *k1,
                                                 const double *sqrtm, const double *isqrtm, int n, int RB, double a,
                                                 const double *x, double *y) {
    // as k_prior: 256 / RB rows per block and pass; wave-uniform rows for RB >= 64
    const int rpb = 256 / RB, r = int(threadIdx.x) % RB, lr = int(threadIdx.x) / RB;
    auto row = [&](int i, bool wave_row) {
        double acc = 0.0;
        if (wave_row) {
            acc = k1_row_wave<true>(rowptr, col, k1, isqrtm, i, RB, r, x);
        } else {
#pragma unroll 4
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int j = col[k];
                acc = __builtin_fma(k1[k], isqrtm[j] * x[int64_t(j) * RB + r], acc);
            }
        }
        const int64_t e = int64_t(i) * RB + r;
        y[e] = sqrtm[i] * x[e] + a * acc;
    };
    for (int64_t i = int64_t(blockIdx.x) * rpb + lr; i < n; i += int64_t(gridDim.x) * rpb) {
        if (RB >= 64) row(__builtin_amdgcn_readfirstlane(int(i)), true);
        else row(int(i), false);
    }
}

// part[b][r] = sum over rows of block b of x[row][r] * y[row][r]
__global__ void __launch_bounds__(256) k_dot_partial(const double *x, const double *y, int64_t rows, int RB,
                                                     double *part) {
    __shared__ double red[256];
    const int G = 256 / RB;
    const int r = threadIdx.x % RB, g = threadIdx.x / RB;
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t a0 = int64_t(blockIdx.x) * chunk, a1 = a0 + chunk < rows ? a0 + chunk : rows;
    // four rows per pass into four partial sums, so that each lane keeps four loads
    // in flight; a norm (x == y) loads each element once
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int64_t row = a0 + g;
    if (x == y) {
        for (; row + 3 * G < a1; row += 4 * G) {
            const double v0 = x[row * RB + r], v1 = x[(row + G) * RB + r], v2 = x[(row + 2 * G) * RB + r],
                         v3 = x[(row + 3 * G) * RB + r];
            acc0 = __builtin_fma(v0, v0, acc0);
            acc1 = __builtin_fma(v1, v1, acc1);
            acc2 = __builtin_fma(v2, v2, acc2);
            acc3 = __builtin_fma(v3, v3, acc3);
        }
    } else {
        for (; row + 3 * G < a1; row += 4 * G) {
            const int64_t e0 = row * RB + r, e1 = e0 + int64_t(G) * RB, e2 = e1 + int64_t(G) * RB,
                          e3 = e2 + int64_t(G) * RB;
            acc0 = __builtin_fma(x[e0], y[e0], acc0);
            acc1 = __builtin_fma(x[e1], y[e1], acc1);
            acc2 = __builtin_fma(x[e2], y[e2], acc2);
            acc3 = __builtin_fma(x[e3], y[e3], acc3);
        }
    }
    for (; row < a1; row += G) {
        const int64_t e = row * RB + r;
        acc0 = __builtin_fma(x[e], y[e], acc0);
    }
    red[threadIdx.x] = (acc0 + acc1) + (acc2 + acc3);
    __syncthreads();
    for (int s = 128; s >= RB; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < RB) part[int64_t(blockIdx.x) * RB + threadIdx.x] = red[threadIdx.x];
}

// part[b][r] = sum over rows of block b of (a[row][aoff + r] - y[row][r])^2, a with row
// stride lda, y with row stride RB (same reduction shape as k_dot_partial)
__global__ void __launch_bounds__(256) k_diff_sq_partial(const double *a, int lda, int aoff, const double *y,
                                                         int64_t rows, int RB, double *part) {
    __shared__ double red[256];
    const int G = 256 / RB;
    const int r = threadIdx.x % RB, g = threadIdx.x / RB;
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t a0 = int64_t(blockIdx.x) * chunk, a1 = a0 + chunk < rows ? a0 + chunk : rows;
    double acc = 0.0;
    for (int64_t row = a0 + g; row < a1; row += G) {
        const double d = a[row * lda + aoff + r] - y[row * RB + r];
        acc = __builtin_fma(d, d, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= RB; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < RB) part[int64_t(blockIdx.x) * RB + threadIdx.x] = red[threadIdx.x];
}

// out[row][r] = in[row][c0 + r], r < RB (in with row stride ldin)
__global__ void k_cols(const double *in, int ldin, int c0, double *out, int64_t total, int RB) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x)
        out[e] = in[(e / RB) * ldin + c0 + e % RB];
}

// out[r] = sum_b partA[b][r] (+ sum_b partB[b][r]), nb partial blocks each
__global__ void __launch_bounds__(256) k_dot_final(const double *partA, const double *partB, int nb, int RB,
                                                   double *out) {
    __shared__ double red[256];
    const int G = 256 / RB;
    const int r = threadIdx.x % RB, g = threadIdx.x / RB;
    double acc = 0.0;
    for (int b = g; b < nb; b += G) acc += partA[int64_t(b) * RB + r];
    if (partB)
        for (int b = g; b < nb; b += G) acc += partB[int64_t(b) * RB + r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= RB; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < RB) out[threadIdx.x] = red[threadIdx.x];
}

__global__ void k_alpha(const double *gamma, const double *delta, double *alpha, int RB) {
    const int r = threadIdx.x;
    if (r < RB) alpha[r] = delta[r] > 0.0 ? gamma[r] / delta[r] : 0.0;
}

__global__ void k_gamma(double *gamma, const double *gnew, double *beta, double *invn, int first, int RB) {
    const int r = threadIdx.x;
    if (r >= RB) return;
    const double g = gnew[r];
    beta[r] = (first || !(gamma[r] > 0.0)) ? 0.0 : g / gamma[r];
    invn[r] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
    gamma[r] = g;
}

__global__ void k_resid(const double *a, const double *b, double *hist, double *diag, int64_t ld, int64_t col,
                        int64_t rb0, int64_t R, int RB) {
    const int r = threadIdx.x;
    if (r >= RB || rb0 + r >= R) return;
    const int64_t at = (rb0 + r) * ld + col;
    if (hist) hist[at] = sqrt(a[r] + b[r]);
    if (diag) {
        diag[2 * at] = sqrt(a[r]);
        diag[2 * at + 1] = sqrt(b[r]);
    }
}

// Grid-stride loops over [rows][RB] arrays: the RHS index of a thread's elements,
// fixed when the stride is a multiple of RB (RB a power of two <= the block size),
// so that no element pays a 64-bit division.
struct RhsIndex {
    int64_t stride;
    int r0, RB;
    bool fixed;
    __device__ RhsIndex(int rb) : RB(rb) {
        stride = int64_t(gridDim.x) * blockDim.x;
        r0 = int((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) % rb);
        fixed = stride % rb == 0;
    }
    __device__ int operator()(int64_t e) const { return fixed ? r0 : int(e % RB); }
};

__global__ void k_update_xr(double *x, const double *d, double *rp, const double *qp, const double *alpha,
                            int64_t total, int RB) {
    const RhsIndex rix(RB);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += rix.stride) {
        const double al = alpha[rix(e)];
        x[e] += al * d[e];
        rp[e] -= al * qp[e];
    }
}

__global__ void k_axpy_neg(double *y, const double *x, const double *alpha, int64_t total, int RB) {
    const RhsIndex rix(RB);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += rix.stride)
        y[e] -= alpha[rix(e)] * x[e];
}

__global__ void k_append(const double *sv, double *Qk, double *d, const double *invn, const double *beta, int first,
                         int64_t total, int RB) {
    const RhsIndex rix(RB);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += rix.stride) {
        const int r = rix(e);
        const double s = sv[e];
        if (Qk) Qk[e] = s * invn[r];
        d[e] = first ? s : s + beta[r] * d[e];
    }
}

// ---- LSQR (Golub-Kahan bidiagonalisation) ---------------------------------
// Per-RHS scalar stages; one thread per right-hand side.  A new alpha or beta
// below 1e-15 of its first value is exact breakdown and is set to zero.
__global__ void k_lsqr_scalar(LsqrStage st, LsqrScalars c, const double *n1, const double *n2, int RB) {
    const int r = threadIdx.x;
    if (r >= RB) return;
    const double nrm = sqrt(n1[r] + (n2 ? n2[r] : 0.0));
    switch (st) {
    case LsqrStage::InitBeta:
        c.beta[r] = c.beta1[r] = nrm;
        c.inv[r] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        break;
    case LsqrStage::InitAlpha:
        c.alpha[r] = c.alpha1[r] = nrm;
        c.inv[r] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        c.phib[r] = c.beta[r];
        c.rhob[r] = nrm;
        c.zfac[r] = 0.0;
        break;
    case LsqrStage::Beta: {
        const double be = nrm > 1e-15 * c.beta1[r] ? nrm : 0.0;
        c.beta[r] = be;
        c.inv[r] = be > 0.0 ? 1.0 / be : 0.0;
        // plane rotation eliminating beta_{k+1} below rho_bar_k
        const double rb = c.rhob[r];
        const double rho = sqrt(rb * rb + be * be);
        const double cs = rho > 0.0 ? rb / rho : 1.0, sn = rho > 0.0 ? be / rho : 0.0;
        const double phi = cs * c.phib[r];
        c.rho[r] = rho;
        c.cs[r] = cs;
        c.sn[r] = sn;
        c.phib[r] = sn * c.phib[r];
        c.step[r] = rho > 0.0 ? phi / rho : 0.0;
        break;
    }
    case LsqrStage::Alpha: {
        const double al = nrm > 1e-15 * c.alpha1[r] ? nrm : 0.0;
        c.alpha[r] = al;
        c.inv[r] = al > 0.0 ? 1.0 / al : 0.0;
        c.rhob[r] = -c.cs[r] * al;
        c.zfac[r] = c.rho[r] > 0.0 ? c.sn[r] * al / c.rho[r] : 0.0;
        break;
    }
    }
}

// out = (sa * ca[r]) a + (sb * cb[r]) b; a null coefficient pointer means 1, b may be null.
__global__ void k_lincomb(double *out, const double *a, const double *ca, double sa, const double *b, const double *cb,
                          double sb, int64_t total, int RB) {
    const RhsIndex rix(RB);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += rix.stride) {
        const int r = rix(e);
        double v = sa * (ca ? ca[r] : 1.0) * a[e];
        if (b) v += sb * (cb ? cb[r] : 1.0) * b[e];
        out[e] = v;
    }
}

// v = inv * sv ; w = v - zfac * w (w = v on the first call) ; Qk = v
__global__ void k_lsqr_vw(const double *sv, const double *inv, const double *zfac, double *v, double *w, double *Qk,
                          int first, int64_t total, int RB) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        const int r = int(e % RB);
        const double vv = inv[r] * sv[e];
        v[e] = vv;
        w[e] = first ? vv : vv - zfac[r] * w[e];
        if (Qk) Qk[e] = vv;
    }
}

// part[b][j][r] = sum over the rows of block b of Q[j][row][r] s[row][r] for j < k, and
// part[b][k + j][r] the same with the newest basis vector Q[k-1] in place of s: the
// first Gram-Schmidt coefficients and the new row of the Gram matrix in one read of Q.
__global__ void __launch_bounds__(256) k_multidot2_partial(const double *Q, const double *sv, int k, int64_t rows,
                                                           int RB, double *part) {
    __shared__ double red[256];
    const int G = 256 / RB;
    const int r = threadIdx.x % RB, g = threadIdx.x / RB;
    const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
    const int64_t a0 = int64_t(blockIdx.x) * chunk, a1 = a0 + chunk < rows ? a0 + chunk : rows;
    const int64_t stride = rows * RB;
    const double *w = Q + int64_t(k - 1) * stride;
    for (int j0 = 0; j0 < k; j0 += 8) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gac[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t row = a0 + g; row < a1; row += G) {
            const int64_t e = row * RB + r;
            const double s = sv[e], q = w[e];
#pragma unroll
            for (int jj = 0; jj < 8; ++jj)
                if (j0 + jj < k) {
                    const double qj = Q[int64_t(j0 + jj) * stride + e];
                    acc[jj] = __builtin_fma(qj, s, acc[jj]);
                    gac[jj] = __builtin_fma(qj, q, gac[jj]);
                }
        }
        for (int h = 0; h < 2; ++h)
            for (int jj = 0; jj < 8 && j0 + jj < k; ++jj) {
                red[threadIdx.x] = h ? gac[jj] : acc[jj];
                __syncthreads();
                for (int s = 128; s >= RB; s >>= 1) {
                    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
                    __syncthreads();
                }
                if (threadIdx.x < RB)
                    part[(int64_t(blockIdx.x) * 2 * k + h * k + j0 + jj) * RB + threadIdx.x] = red[threadIdx.x];
                __syncthreads();
            }
    }
}

// Second Gram-Schmidt pass from the Gram matrix, one thread per right-hand side.
// cg[j] (j < k) are the first-pass coefficients c1 = Q^T s, cg[k + j] = Q_j . Q_{k-1}.
// Stores that row into gram ([kcap][kcap][RB], symmetric) and writes
//   coef = c1 + c2,  c2 = Q^T (s - Q c1) = c1 - (Q^T Q) c1,
// so that s - Q coef equals two classical Gram-Schmidt passes in exact arithmetic.
__global__ void k_gram_coef(double *gram, int kcap, const double *cg, int k, int RB, double *coef) {
    const int r = threadIdx.x;
    if (r >= RB) return;
    for (int j = 0; j < k; ++j) {
        const double v = cg[int64_t(k + j) * RB + r];
        gram[(int64_t(k - 1) * kcap + j) * RB + r] = v;
        gram[(int64_t(j) * kcap + (k - 1)) * RB + r] = v;
    }
    for (int j = 0; j < k; ++j) {
        double gc = 0.0;
        for (int i = 0; i < k; ++i) gc = __builtin_fma(gram[(int64_t(j) * kcap + i) * RB + r], cg[int64_t(i) * RB + r], gc);
        const double c1 = cg[int64_t(j) * RB + r];
        coef[int64_t(j) * RB + r] = c1 + (c1 - gc);
    }
}

// coef[j][r] = sum_b part[b][j][r]; one workgroup per j
__global__ void __launch_bounds__(256) k_multidot_final(const double *part, int nb, int k, int RB, double *coef) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    const int G = 256 / RB;
    const int r = threadIdx.x % RB, g = threadIdx.x / RB;
    double acc = 0.0;
    for (int b = g; b < nb; b += G) acc += part[(int64_t(b) * k + j) * RB + r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= RB; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < RB) coef[int64_t(j) * RB + threadIdx.x] = red[threadIdx.x];
}

// s[row][r] -= coef[j][r] * Q[j][row][r], j = 0..k-1 in order
__global__ void k_project(const double *Q, double *sv, const double *coef, int k, int64_t rows, int RB) {
    const int64_t total = rows * RB;
    const RhsIndex rix(RB);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += rix.stride) {
        const int r = rix(e);
        double s = sv[e];
        for (int j = 0; j < k; ++j) s -= coef[int64_t(j) * RB + r] * Q[int64_t(j) * total + e];
        sv[e] = s;
    }
}

__global__ void k_stats(const double *x, int64_t S, int64_t N, double *mean, double *std) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
        double m = 0.0;
        for (int64_t s = 0; s < S; ++s) m += x[s * N + i];
        m /= double(S);
        double v = 0.0;
        for (int64_t s = 0; s < S; ++s) {
            const double d = x[s * N + i] - m;
            v = __builtin_fma(d, d, v);
        }
        if (mean) mean[i] = m;
        if (std) std[i] = S > 1 ? sqrt(v / double(S - 1)) : 0.0;
    }
}

// Convergence diagnostics of one sample per thread from its (||r_d||, ||r_p||) history.
__global__ void k_diagnostics(const double *diag, int64_t S, int n_it, double sqrt_nd, double tau, double *data,
                              double *prior, double *ext, int32_t *first) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const double *h = diag + k * int64_t(n_it) * 2;
    const double b0 = sqrt(h[0] * h[0] + h[1] * h[1]);
    const double ib = b0 > 0.0 ? 1.0 / b0 : 1.0;
    int32_t hit = -1;
    for (int j = 0; j < n_it; ++j) {
        const double nd = h[2 * j], np = h[2 * j + 1];
        if (data) data[k * n_it + j] = nd / sqrt_nd;
        if (prior) prior[k * n_it + j] = np * ib;
        if (ext) ext[k * n_it + j] = sqrt(nd * nd + np * np) * ib;
        if (hit < 0 && nd <= tau * sqrt_nd) hit = j;
    }
    if (first) first[k] = hit;
}

int grid_for(int64_t total, int per_block = 256, int cap = 65536) {
    int64_t g = (total + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return int(g < cap ? g : cap);
}

template <typename T>
RowOps<T> row_ops(const DevOps &op);
template <>
RowOps<double> row_ops<double>(const DevOps &op) {
    return RowOps<double>{op.ell_col, op.xptr, op.xcol, op.bsoff, op.ell_val64, op.xval64, op.bslot64, op.dtm64,
                          op.bnum};
}
template <>
RowOps<float> row_ops<float>(const DevOps &op) {
    return RowOps<float>{op.ell_col, op.xptr, op.xcol, op.bsoff, op.ell_val32, op.xval32, op.bslot32, op.dtm32,
                         op.bnum};
}
template <typename T>
const T *sw_of(const DevOps &op);
template <>
const double *sw_of<double>(const DevOps &op) { return op.sw64; }
template <>
const float *sw_of<float>(const DevOps &op) { return op.sw32; }
template <typename T>
const T *injw_of(const DevOps &op);
template <>
const double *injw_of<double>(const DevOps &op) { return op.injw64; }
template <>
const float *injw_of<float>(const DevOps &op) { return op.injw32; }

// bytes of a step's state (two vectors read, one written) for one RHS block
inline double state_bytes(const DevOps &op, int RB, size_t tsize) { return 3.0 * op.n * RB * double(tsize); }

template <typename T, int RB>
VFwdArgs<T> fwd_args_v(const DevOps &op, const void *S, const void *Sp, void *Sn, bool rows, bool sample, int t,
                       void *y, double yscale, int *blocks) {
    using G = VGeo<T, RB>;
    VFwdArgs<T> a;
    a.o = row_ops<T>(op);
    a.snode = op.snode;
    a.sw = sw_of<T>(op);
    a.S = static_cast<const T *>(S); a.Sp = static_cast<const T *>(Sp); a.Sn = static_cast<T *>(Sn);
    a.y = y; a.yscale = yscale;
    a.n = op.n; a.n_obs = op.n_obs;
    a.n_tiles = rows ? (op.n + G::RPB - 1) / G::RPB : 0;
    a.sample = sample; a.t = t;
    a.dt = T(op.dt);
    a.n_samp = sample ? int((int64_t(op.n_obs) * RB + 255) / 256) : 0;
    a.stream = state_bytes(op, RB, sizeof(T)) > kInfinityCacheBytes;
    a.hdesc = op.ht_desc; a.hrow = op.ht_hrow; a.hmeta = op.ht_meta; a.n_ht = op.n_ht;
    *blocks = a.n_tiles + a.n_samp;
    return a;
}

// workgroups of a halo kernel launch: as many per CU as the LDS allows, a multiple of the 8 XCDs
inline int halo_grid(const DevOps &op) { return (kHPerCU * op.n_cu + 7) / 8 * 8; }

// the halo kernels take float32 blocks of 256-byte row chunks (rows == false:
// a sampling-only launch stays with the vector-lane kernel)
template <typename T, int RB>
bool use_halo(const DevOps &op, bool rows) {
    return std::is_same<T, float>::value && RB >= 64 && RB <= 256 && rows && op.n_ht > 0 && op.n_cu > 0;
}

template <typename T, typename OT, int RB>
void fwd_impl_v(const DevOps &op, const void *S, const void *Sp, void *Sn, bool rows, bool sample, int t, void *y,
                double yscale, hipStream_t s) {
    int grid = 0;
    const VFwdArgs<T> a = fwd_args_v<T, RB>(op, S, Sp, Sn, rows, sample, t, y, yscale, &grid);
    if (grid <= 0) return;
    if constexpr (std::is_same<T, float>::value && RB >= 64 && RB <= 256) {
        if (use_halo<T, RB>(op, rows)) {
            if (a.stream) hipLaunchKernelGGL((k_fwd_h<OT, RB, true>), dim3(halo_grid(op)), dim3(kHThreads), 0, s, a);
            else hipLaunchKernelGGL((k_fwd_h<OT, RB, false>), dim3(halo_grid(op)), dim3(kHThreads), 0, s, a);
            return;
        }
    }
    if (a.stream) hipLaunchKernelGGL((k_fwd_v<T, OT, RB, true>), dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_fwd_v<T, OT, RB, false>), dim3(grid), dim3(256), 0, s, a);
}

template <typename T, typename OT, int RB>
void fwd_impl_vm(const FwdStep *st, int n, hipStream_t s) {
    Multi<VFwdArgs<T>> mm{};
    for (int m = 0; m < n; ++m)
        mm.a[m] = fwd_args_v<T, RB>(*st[m].op, st[m].S, st[m].Sp, st[m].Sn, st[m].rows, st[m].sample, st[m].t,
                                    st[m].y, st[m].yscale, &mm.tiles[m]);
    mm.n = n;
    double sb = 0.0;
    for (int m = 0; m < n; ++m) sb += state_bytes(*st[m].op, RB, sizeof(T));
    const int grid = multi_grid(mm.tiles, n);
    if (grid <= 0) return;
    if (sb > kInfinityCacheBytes) hipLaunchKernelGGL((k_fwd_vm<T, OT, RB, true>), dim3(grid), dim3(256), 0, s, mm);
    else hipLaunchKernelGGL((k_fwd_vm<T, OT, RB, false>), dim3(grid), dim3(256), 0, s, mm);
}

template <typename T, int RB>
VAdjArgs<T> adj_args_v(const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int tb, const void *yh,
                       double yscale) {
    using G = VGeo<T, RB>;
    VAdjArgs<T> a;
    a.o = row_ops<T>(op);
    a.injptr = op.injptr; a.injs = op.injs;
    a.injw = injw_of<T>(op);
    a.S = static_cast<const T *>(S); a.Sp = static_cast<const T *>(Sp); a.Sn = static_cast<T *>(Sn);
    a.yh = yh; a.yscale = yscale;
    a.n = op.n; a.n_obs = op.n_obs; a.last = last;
    a.tb = tb; a.ta = last ? -1 : tb + 1;
    a.n_tiles = (op.n + G::RPB - 1) / G::RPB;
    a.dt = T(op.dt);
    a.stream = state_bytes(op, RB, sizeof(T)) > kInfinityCacheBytes;
    a.hdesc = op.ht_desc; a.hrow = op.ht_hrow; a.hmeta = op.ht_meta; a.n_ht = op.n_ht;
    return a;
}

template <typename T, typename YT, int RB>
void adj_impl_v(const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int tb, const void *yh,
                double yscale, hipStream_t s) {
    const VAdjArgs<T> a = adj_args_v<T, RB>(op, S, Sp, Sn, last, tb, yh, yscale);
    if constexpr (std::is_same<T, float>::value && RB >= 64 && RB <= 256) {
        if (use_halo<T, RB>(op, true)) {
            const dim3 g(halo_grid(op)), b(kHThreads);
            if (a.stream) {
                if (last) hipLaunchKernelGGL((k_adj_h<YT, RB, true, true>), g, b, 0, s, a);
                else hipLaunchKernelGGL((k_adj_h<YT, RB, true, false>), g, b, 0, s, a);
            } else {
                if (last) hipLaunchKernelGGL((k_adj_h<YT, RB, false, true>), g, b, 0, s, a);
                else hipLaunchKernelGGL((k_adj_h<YT, RB, false, false>), g, b, 0, s, a);
            }
            return;
        }
    }
    if (a.stream) hipLaunchKernelGGL((k_adj_v<T, YT, RB, true>), dim3(a.n_tiles), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_adj_v<T, YT, RB, false>), dim3(a.n_tiles), dim3(256), 0, s, a);
}

template <typename T, typename YT, int RB>
void adj_impl_vm(const AdjStep *st, int n, hipStream_t s) {
    Multi<VAdjArgs<T>> mm{};
    for (int m = 0; m < n; ++m) {
        mm.a[m] = adj_args_v<T, RB>(*st[m].op, st[m].S, st[m].Sp, st[m].Sn, st[m].last, st[m].tb, st[m].yh,
                                    st[m].yscale);
        mm.tiles[m] = mm.a[m].n_tiles;
    }
    mm.n = n;
    double sb = 0.0;
    for (int m = 0; m < n; ++m) sb += state_bytes(*st[m].op, RB, sizeof(T));
    const int grid = multi_grid(mm.tiles, n);
    if (grid <= 0) return;
    if (sb > kInfinityCacheBytes) hipLaunchKernelGGL((k_adj_vm<T, YT, RB, true>), dim3(grid), dim3(256), 0, s, mm);
    else hipLaunchKernelGGL((k_adj_vm<T, YT, RB, false>), dim3(grid), dim3(256), 0, s, mm);
}

template <typename T, typename OT, int RB>
void fwd_impl(const DevOps &op, const void *S, const void *Sp, void *Sn, bool rows, bool sample, int t, void *y,
              double yscale, hipStream_t s) {
    if constexpr (RB * sizeof(T) >= 16) {
        // a row of the RHS block fits one wave (64 lanes x 16 bytes): up to 256 float / 128 double
        if constexpr (RB * sizeof(T) <= 1024) fwd_impl_v<T, OT, RB>(op, S, Sp, Sn, rows, sample, t, y, yscale, s);
    } else {
        using G = Geo<RB>;
        FwdArgs<T> a;
        a.o = row_ops<T>(op);
        a.snode = op.snode;
        a.sw = sw_of<T>(op);
        a.S = static_cast<const T *>(S); a.Sp = static_cast<const T *>(Sp); a.Sn = static_cast<T *>(Sn);
        a.y = y; a.yscale = yscale;
        a.n = op.n; a.n_obs = op.n_obs;
        a.n_tiles = rows ? (op.n + G::RPB - 1) / G::RPB : 0;
        a.sample = sample; a.t = t;
        a.dt = T(op.dt);
        a.n_samp = sample ? int((int64_t(op.n_obs) * RB + 255) / 256) : 0;
        const int grid = a.n_tiles + a.n_samp;
        if (grid > 0) hipLaunchKernelGGL((k_fwd<T, OT, RB>), dim3(grid), dim3(256), 0, s, a);
    }
}

template <typename T, typename YT, int RB>
AdjArgs<T> adj_args(const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int ta, int tb,
                    const void *yh, double yscale) {
    using G = Geo<RB * sizeof(T) >= 16 ? 1 : RB>;  // the scalar-lane geometry, used only below 16 bytes per row
    AdjArgs<T> a;
    a.o = row_ops<T>(op);
    a.injptr = op.injptr; a.injs = op.injs;
    a.injw = injw_of<T>(op);
    a.S = static_cast<const T *>(S); a.Sp = static_cast<const T *>(Sp); a.Sn = static_cast<T *>(Sn);
    a.yh = yh; a.yscale = yscale;
    a.n = op.n; a.n_obs = op.n_obs; a.last = last; a.ta = ta; a.tb = tb;
    a.n_tiles = (op.n + G::RPB - 1) / G::RPB;
    a.dt = T(op.dt);
    return a;
}

template <typename T, typename YT, int RB>
void adj_impl(const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int tb, const void *yh,
              double yscale, hipStream_t s) {
    if constexpr (RB * sizeof(T) >= 16) {
        if constexpr (RB * sizeof(T) <= 1024) adj_impl_v<T, YT, RB>(op, S, Sp, Sn, last, tb, yh, yscale, s);
    } else {
        const AdjArgs<T> a = adj_args<T, YT, RB>(op, S, Sp, Sn, last, last ? -1 : tb + 1, tb, yh, yscale);
        hipLaunchKernelGGL((k_adj<T, YT, RB>), dim3(a.n_tiles), dim3(256), 0, s, a);
    }
}

template <typename T, typename YT, int RB>
void adj_init(const DevOps &op, void *q0, void *qm1, const void *yh, double yscale, hipStream_t s) {
    const AdjArgs<T> a = adj_args<T, YT, RB>(op, nullptr, nullptr, nullptr, false, -1, op.n_steps - 1, yh, yscale);
    hipLaunchKernelGGL((k_adj_init<T, YT, RB>), dim3(grid_for(int64_t(op.n) * RB)), dim3(256), 0, s, a,
                       static_cast<T *>(q0), static_cast<T *>(qm1));
}

template <typename T, typename OT, int RB>
void fwd_multi(const FwdStep *st, int n, hipStream_t s) {
    if constexpr (RB * sizeof(T) >= 16 && RB * sizeof(T) <= 1024) fwd_impl_vm<T, OT, RB>(st, n, s);
}
template <typename T, typename YT, int RB>
void adj_multi(const AdjStep *st, int n, hipStream_t s) {
    if constexpr (RB * sizeof(T) >= 16 && RB * sizeof(T) <= 1024) adj_impl_vm<T, YT, RB>(st, n, s);
}

#define PAT_RB_SWITCH(RBV, CALL)               \
    switch (RBV) {                             \
        case 1: { constexpr int RB_ = 1; CALL; break; }   \
        case 2: { constexpr int RB_ = 2; CALL; break; }   \
        case 4: { constexpr int RB_ = 4; CALL; break; }   \
        case 8: { constexpr int RB_ = 8; CALL; break; }   \
        case 16: { constexpr int RB_ = 16; CALL; break; } \
        case 32: { constexpr int RB_ = 32; CALL; break; } \
        case 64: { constexpr int RB_ = 64; CALL; break; } \
        case 128: { constexpr int RB_ = 128; CALL; break; } \
        case 256: { constexpr int RB_ = 256; CALL; break; } \
        default: break;                                   \
    }

}  // namespace

void launch_fwd_step(Prec prec, int RB, const DevOps &op, const void *S, const void *Sp, void *Sn, bool rows,
                     bool sample, int t, void *y, bool y_is_f64, double yscale, hipStream_t s) {
    if (prec == Prec::F64) {
        PAT_RB_SWITCH(RB, (fwd_impl<double, double, RB_>(op, S, Sp, Sn, rows, sample, t, y, yscale, s)));
    } else if (y_is_f64) {
        PAT_RB_SWITCH(RB, (fwd_impl<float, double, RB_>(op, S, Sp, Sn, rows, sample, t, y, yscale, s)));
    } else {
        PAT_RB_SWITCH(RB, (fwd_impl<float, float, RB_>(op, S, Sp, Sn, rows, sample, t, y, yscale, s)));
    }
}

void launch_adj_init(Prec prec, int RB, const DevOps &op, void *q0, void *qm1, const void *yhat, bool y_is_f64,
                     double yscale, hipStream_t s) {
    if (prec == Prec::F64) {
        PAT_RB_SWITCH(RB, (adj_init<double, double, RB_>(op, q0, qm1, yhat, yscale, s)));
    } else if (y_is_f64) {
        PAT_RB_SWITCH(RB, (adj_init<float, double, RB_>(op, q0, qm1, yhat, yscale, s)));
    } else {
        PAT_RB_SWITCH(RB, (adj_init<float, float, RB_>(op, q0, qm1, yhat, yscale, s)));
    }
}

void launch_adj_step(Prec prec, int RB, const DevOps &op, const void *S, const void *Sp, void *Sn, bool last, int tb,
                     const void *yhat, bool y_is_f64, double yscale, hipStream_t s) {
    if (prec == Prec::F64) {
        PAT_RB_SWITCH(RB, (adj_impl<double, double, RB_>(op, S, Sp, Sn, last, tb, yhat, yscale, s)));
    } else if (y_is_f64) {
        PAT_RB_SWITCH(RB, (adj_impl<float, double, RB_>(op, S, Sp, Sn, last, tb, yhat, yscale, s)));
    } else {
        PAT_RB_SWITCH(RB, (adj_impl<float, float, RB_>(op, S, Sp, Sn, last, tb, yhat, yscale, s)));
    }
}

bool multi_step_supported(Prec prec, int RB) { return RB * (prec == Prec::F64 ? 8 : 4) >= 16; }

int max_rhs_block(Prec prec) { return prec == Prec::F64 ? 128 : 256; }

void launch_fwd_multi(Prec prec, int RB, bool y_is_f64, const FwdStep *st, int n, hipStream_t s) {
    if (prec == Prec::F64) {
        PAT_RB_SWITCH(RB, (fwd_multi<double, double, RB_>(st, n, s)));
    } else if (y_is_f64) {
        PAT_RB_SWITCH(RB, (fwd_multi<float, double, RB_>(st, n, s)));
    } else {
        PAT_RB_SWITCH(RB, (fwd_multi<float, float, RB_>(st, n, s)));
    }
}

void launch_adj_multi(Prec prec, int RB, bool y_is_f64, const AdjStep *st, int n, hipStream_t s) {
    if (prec == Prec::F64) {
        PAT_RB_SWITCH(RB, (adj_multi<double, double, RB_>(st, n, s)));
    } else if (y_is_f64) {
        PAT_RB_SWITCH(RB, (adj_multi<float, double, RB_>(st, n, s)));
    } else {
        PAT_RB_SWITCH(RB, (adj_multi<float, float, RB_>(st, n, s)));
    }
}

void launch_pack(bool in_f64, bool out_f64, const void *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                 const int32_t *perm, void *out, hipStream_t s) {
    const dim3 g(unsigned((cols + 63) / 64)), b(256);
    if (in_f64 && out_f64)
        hipLaunchKernelGGL((k_pack<double, double>), g, b, 0, s, (const double *)in, R, rb0, RB, cols, perm, (double *)out);
    else if (in_f64)
        hipLaunchKernelGGL((k_pack<double, float>), g, b, 0, s, (const double *)in, R, rb0, RB, cols, perm, (float *)out);
    else if (out_f64)
        hipLaunchKernelGGL((k_pack<float, double>), g, b, 0, s, (const float *)in, R, rb0, RB, cols, perm, (double *)out);
    else
        hipLaunchKernelGGL((k_pack<float, float>), g, b, 0, s, (const float *)in, R, rb0, RB, cols, perm, (float *)out);
}

void launch_unpack(bool in_f64, bool out_f64, const void *in, int64_t R, int64_t rb0, int RB, int64_t cols,
                   const int32_t *perm, void *out, hipStream_t s) {
    const dim3 g(unsigned((cols + 63) / 64)), b(256);
    if (in_f64 && out_f64)
        hipLaunchKernelGGL((k_unpack<double, double>), g, b, 0, s, (const double *)in, R, rb0, RB, cols, perm, (double *)out);
    else if (in_f64)
        hipLaunchKernelGGL((k_unpack<double, float>), g, b, 0, s, (const double *)in, R, rb0, RB, cols, perm, (float *)out);
    else if (out_f64)
        hipLaunchKernelGGL((k_unpack<float, double>), g, b, 0, s, (const float *)in, R, rb0, RB, cols, perm, (double *)out);
    else
        hipLaunchKernelGGL((k_unpack<float, float>), g, b, 0, s, (const float *)in, R, rb0, RB, cols, perm, (float *)out);
}

void launch_fill(double *x, int64_t count, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(256), 0, s, x, count, v);
}

void launch_cast_to_state(Prec prec, const double *x, void *P, int64_t count, hipStream_t s) {
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_cast<double>), dim3(grid_for(count)), dim3(256), 0, s, x, (double *)P, count);
    else
        hipLaunchKernelGGL((k_cast<float>), dim3(grid_for(count)), dim3(256), 0, s, x, (float *)P, count);
}

void launch_normals(uint64_t seed, int kind, int64_t k0, int64_t S, int64_t len, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_normals, dim3(grid_for(S * ((len + 3) / 4))), dim3(256), 0, s, seed, kind, k0, S, len, out);
}
void launch_build_rhs_rng(const double *yobs, uint64_t seed, int64_t k0, int64_t S, int64_t rb0, int RB, int64_t M,
                          double isig, double *bd, hipStream_t s) {
    hipLaunchKernelGGL(k_build_rhs_rng, dim3(grid_for(((M + 3) / 4) * RB)), dim3(256), 0, s, yobs, seed, k0, S, rb0, RB,
                       M, isig, bd);
}
void launch_xi_rng(uint64_t seed, int64_t k0, int64_t S, int64_t rb0, int RB, int64_t N, const int32_t *perm,
                   double *xi, hipStream_t s) {
    hipLaunchKernelGGL(k_xi_rng, dim3(grid_for(N * RB)), dim3(256), 0, s, seed, k0, S, rb0, RB, N, perm, xi);
}
void launch_build_rhs(const double *yobs, const double *eta, int64_t S, int64_t rb0, int RB, int64_t M, double isig,
                      double *bd, hipStream_t s) {
    hipLaunchKernelGGL(k_build_rhs, dim3(unsigned((M + 63) / 64)), dim3(256), 0, s, yobs, eta, S, rb0, RB, M, isig, bd);
}

// (the prior kernels take RB a power of two <= 256, as every RHS block is)
void launch_prior(const DevOps &op, int RB, double a, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_prior, dim3(grid_for(int64_t(op.n) * RB)), dim3(256), 0, s, op.rowptr, op.col, op.k1val64,
                       op.sqrtm, op.isqrtm, op.n, RB, a, x, y);
}

void launch_prior_t(const DevOps &op, int RB, double a, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_prior_t, dim3(grid_for(int64_t(op.n) * RB)), dim3(256), 0, s, op.rowptr, op.col, op.k1val64,
                       op.sqrtm, op.isqrtm, op.n, RB, a, x, y);
}

void launch_gext_t_combine(Prec prec, const DevOps &op, int RB, double a, double isig, const void *PH, const double *rp,
                           double *out, hipStream_t s) {
    const dim3 g(grid_for(int64_t(op.n) * RB)), b(256);
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_gext_t<double>), g, b, 0, s, op.rowptr, op.col, op.k1val64, op.sqrtm, op.isqrtm, op.n, RB,
                           a, isig, (const double *)PH, rp, out);
    else
        hipLaunchKernelGGL((k_gext_t<float>), g, b, 0, s, op.rowptr, op.col, op.k1val64, op.sqrtm, op.isqrtm, op.n, RB,
                           a, isig, (const float *)PH, rp, out);
}

void launch_dot_partial(const double *x, const double *y, int64_t rows, int RB, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, x, y, rows, RB, part);
}

void launch_diff_sq_partial(const double *a, int lda, int aoff, const double *y, int64_t rows, int RB, double *part,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_diff_sq_partial, dim3(kDotBlocks), dim3(256), 0, s, a, lda, aoff, y, rows, RB, part);
}

void launch_cols(const double *in, int ldin, int c0, double *out, int64_t rows, int RB, hipStream_t s) {
    hipLaunchKernelGGL(k_cols, dim3(grid_for(rows * RB)), dim3(256), 0, s, in, ldin, c0, out, rows * RB, RB);
}

void launch_dot_final(const double *partA, const double *partB, int RB, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, partA, partB, kDotBlocks, RB, out);
}

void launch_scalar_alpha(const double *gamma, const double *delta, double *alpha, int RB, hipStream_t s) {
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(256), 0, s, gamma, delta, alpha, RB);
}

void launch_scalar_gamma(double *gamma, const double *gnew, double *beta, double *invn, int first, int RB,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_gamma, dim3(1), dim3(256), 0, s, gamma, gnew, beta, invn, first, RB);
}

void launch_resid(const double *a, const double *b, double *hist, double *diag, int64_t ld, int64_t col, int64_t rb0,
                  int64_t R, int RB, hipStream_t s) {
    hipLaunchKernelGGL(k_resid, dim3(1), dim3(256), 0, s, a, b, hist, diag, ld, col, rb0, R, RB);
}

void launch_lsqr_scalar(LsqrStage st, const LsqrScalars &c, const double *n1, const double *n2, int RB,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(256), 0, s, st, c, n1, n2, RB);
}

void launch_lincomb(double *out, const double *a, const double *ca, double sa, const double *b, const double *cb,
                    double sb, int64_t rows, int RB, hipStream_t s) {
    const int64_t total = rows * RB;
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(total)), dim3(256), 0, s, out, a, ca, sa, b, cb, sb, total, RB);
}

void launch_lsqr_vw(const double *sv, const double *inv, const double *zfac, double *v, double *w, double *Qk,
                    int first, int64_t rows, int RB, hipStream_t s) {
    const int64_t total = rows * RB;
    hipLaunchKernelGGL(k_lsqr_vw, dim3(grid_for(total)), dim3(256), 0, s, sv, inv, zfac, v, w, Qk, first, total, RB);
}

void launch_update_xr(double *x, const double *d, double *rp, const double *qp, const double *alpha, int64_t rows,
                      int RB, hipStream_t s) {
    const int64_t total = rows * RB;
    hipLaunchKernelGGL(k_update_xr, dim3(grid_for(total)), dim3(256), 0, s, x, d, rp, qp, alpha, total, RB);
}

void launch_axpy_neg(double *y, const double *x, const double *alpha, int64_t rows, int RB, hipStream_t s) {
    const int64_t total = rows * RB;
    hipLaunchKernelGGL(k_axpy_neg, dim3(grid_for(total)), dim3(256), 0, s, y, x, alpha, total, RB);
}

void launch_append_dir(const double *sv, double *Qk, double *d, const double *invn, const double *beta, int first,
                       int64_t rows, int RB, hipStream_t s) {
    const int64_t total = rows * RB;
    hipLaunchKernelGGL(k_append, dim3(grid_for(total)), dim3(256), 0, s, sv, Qk, d, invn, beta, first, total, RB);
}

void launch_reorth_coef(const double *Q, const double *sv, int k, int64_t rows, int RB, double *part, double *cg,
                        double *gram, int kcap, double *coef, hipStream_t s) {
    if (k <= 0) return;
    hipLaunchKernelGGL(k_multidot2_partial, dim3(kMultiBlocks), dim3(256), 0, s, Q, sv, k, rows, RB, part);
    hipLaunchKernelGGL(k_multidot_final, dim3(2 * k), dim3(256), 0, s, part, kMultiBlocks, 2 * k, RB, cg);
    hipLaunchKernelGGL(k_gram_coef, dim3(1), dim3(256), 0, s, gram, kcap, cg, k, RB, coef);
}

void launch_project(const double *Q, double *sv, const double *coef, int k, int64_t rows, int RB, hipStream_t s) {
    if (k <= 0) return;
    hipLaunchKernelGGL(k_project, dim3(grid_for(rows * RB)), dim3(256), 0, s, Q, sv, coef, k, rows, RB);
}

void launch_diagnostics(const double *diag, int64_t S, int n_it, int64_t n_data, double tau, double *data,
                        double *prior, double *ext, int32_t *first, hipStream_t s) {
    hipLaunchKernelGGL(k_diagnostics, dim3(grid_for(S)), dim3(256), 0, s, diag, S, n_it, sqrt(double(n_data)), tau,
                       data, prior, ext, first);
}

void launch_stats(const double *samples, int64_t S, int64_t N, double *mean, double *std, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(grid_for(N)), dim3(256), 0, s, samples, S, N, mean, std);
}

}  // namespace pat
