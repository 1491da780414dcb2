// Whittle-Matern Fourier-spectral prior on the GPU (Sec. 4.1.2 eq. (matern-cov-op);
// the construction of Sec. 6.4): p0 = P w with P = I_h F^* diag(a) F, w a latent
// white-noise grid vector, F the 3D DFT on a periodic n^3 box, a(k) the
// square-root spectrum, I_h trilinear interpolation to the mesh nodes.
//
// Layouts: grid vectors [n^3][RB] with grid index g = (k*n + j)*n + i (x fastest)
// and the RHS fastest.  The filtered field is real, so its spectrum is kept only
// for the nh = n/2 + 1 non-negative x frequencies (the others are the complex
// conjugates): complex half-spectrum vectors [n][n][nh][RB], (re, im) per element.
//
// The 3D transform is five launches, each a batch of one-dimensional transforms
// along one axis (one line and a chunk of up to 16 right-hand sides per
// workgroup, staged in LDS): the real-to-complex x pass, forward y, then forward
// z, the multiplication by a(k) and the inverse z in the same pass, inverse y, and
// the complex-to-real x pass.  The x passes pack the n real points of a line as
// n/2 complex points (even samples real, odd samples imaginary), transform those
// with one length-n/2 FFT and split the result into the n/2 + 1 spectrum values
// (and back), which halves the bytes of every pass after the first.  Each complex
// transform is a Stockham FFT (natural order in and out, so no reordering pass)
// with 8 points per thread: radix-8 stages computed in registers, exchanged
// through LDS between stages, then a radix-2 or radix-4 stage when the length is
// not a power of 8 (n = 128: 8 x 8 x 2 along y and z, 8 x 8 along x).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pat_kernels.h"

namespace pat {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conjg(double2 a) { return make_double2(a.x, -a.y); }

constexpr int kRC = 16;  // right-hand sides per workgroup
// elements a thread stages between global memory and LDS at most: n * RC / 256
// (n <= 128 points per line, RC <= 16), all loads issued before any is consumed
constexpr int kPer = 128 * kRC / 256;

enum : int { kForward = 0, kInverse = 1, kCentre = 2 };

struct FftPass {
    const double *rin;   // real input [G][RB] (x pass, forward), or null
    const double2 *cin;  // complex half-spectrum input, or null
    double2 *cout;       // complex half-spectrum output, or null
    double *rout;        // real output (x pass, inverse), or null
    const double *add;   // added to the real output, or null
    const double *amp;   // a(k) for the centre pass, [(ky * nh + kx) * n + kz]: z lines contiguous
    const double2 *tw;   // tw[j] = exp(-2 pi i j / n), j < n/2
    int n, RB, axis, mode;
};

// Radix-2 butterfly (u, t) -> (u + t, u - t).
__device__ __forceinline__ void bfly(double2 &u, double2 &t) {
    const double2 s = cadd(u, t);
    t = csub(u, t);
    u = s;
}
// multiplication by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 rot4(double2 a) { return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x); }

// 8-point DFT in registers, natural order in and out, w = exp(-2 pi i / 8) (forward) or its conjugate.
template <bool INV>
__device__ __forceinline__ void dft8(double2 v[8]) {
    constexpr double h = 0.70710678118654752440;
    double2 a0 = v[0], a1 = v[4], a2 = v[2], a3 = v[6], a4 = v[1], a5 = v[5], a6 = v[3], a7 = v[7];
    bfly(a0, a1); bfly(a2, a3); bfly(a4, a5); bfly(a6, a7);
    a3 = rot4<INV>(a3); a7 = rot4<INV>(a7);
    bfly(a0, a2); bfly(a1, a3); bfly(a4, a6); bfly(a5, a7);
    // w8^1, w8^2, w8^3 on a5, a6, a7
    a5 = INV ? make_double2(h * (a5.x - a5.y), h * (a5.x + a5.y)) : make_double2(h * (a5.x + a5.y), h * (a5.y - a5.x));
    a6 = rot4<INV>(a6);
    a7 = INV ? make_double2(-h * (a7.x + a7.y), h * (a7.x - a7.y)) : make_double2(h * (a7.y - a7.x), -h * (a7.x + a7.y));
    bfly(a0, a4); bfly(a1, a5); bfly(a2, a6); bfly(a3, a7);
    v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3; v[4] = a4; v[5] = a5; v[6] = a6; v[7] = a7;
}

template <bool INV>
__device__ __forceinline__ void dft4(double2 v[4]) {
    double2 a0 = v[0], a1 = v[2], a2 = v[1], a3 = v[3];
    bfly(a0, a1); bfly(a2, a3);
    a3 = rot4<INV>(a3);
    bfly(a0, a2); bfly(a1, a3);
    v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3;
}

// LDS position of point t of a line: one pad element after every 8 points, so the
// stride-8 writes of the first radix-8 stage spread over all LDS banks
__device__ __forceinline__ int pidx(int t) { return t + (t >> 3); }

// w^e, w = exp(-2 pi i / n), from the table of the first n/2 powers (conjugate for the inverse)
template <bool INV>
__device__ __forceinline__ double2 wpow(const double2 *tws, int e, int n) {
    e &= n - 1;
    const int h = n >> 1;
    double2 w = e < h ? tws[e] : make_double2(-tws[e - h].x, -tws[e - h].y);
    return INV ? conjg(w) : w;
}

// One length-n transform (Stockham, natural order in and out) of each of the RC lines
// of a workgroup, 8 points per thread: radix-8 stages while 8^s divides n, then a
// final radix-2 or radix-4 stage.  The first stage takes its points from
// load(line, t) and the last hands its results to store(line, t, value); the stages
// in between exchange through the LDS tile X (line r at X + r * stride, see pidx).
// So a pass reads its input once and writes its output once, with no staging copy
// through LDS.  The first and last stages map thread -> (line = thread % RC,
// j = thread / RC), so that consecutive threads touch consecutive right-hand sides
// of a point in memory.  load may read X and store may write X: every stage reads
// all its inputs and waits at a barrier before it writes.  Threads without a line
// only take part in the barriers.  Ends with a barrier.
template <bool INV, typename Load, typename Store>
__device__ __forceinline__ void line_fft_io(double2 *X, int stride, int n, int RC, const double2 *tws, Load load,
                                            Store store) {
    const int tid = threadIdx.x;
    if (n < 8) {  // n = 2 or 4 (the x passes of a grid of 4 or 8): one thread per line
        double2 v[4];
        const bool act = tid < RC;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double2 x = make_double2(0.0, 0.0);
            if (act && t < n) x = load(tid, t);
            v[t] = x;
        }
        __syncthreads();
        if (act) {
            if (n == 4) dft4<INV>(v);
            else bfly(v[0], v[1]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < n) store(tid, t, v[t]);
        }
        __syncthreads();
        return;
    }
    const int tpl = n >> 3;  // threads per line
    int n8 = 1;              // the radix-8 part: 8^s dividing n
    while (n8 * 8 <= n) n8 *= 8;
    const int rf = n / n8;  // 1, 2 or 4 left for the final stage
    for (int ns = 1; ns < n8; ns *= 8) {
        const bool first = ns == 1, last = ns * 8 == n8 && rf == 1;
        const bool io = first || last;
        const int line = io ? tid % RC : tid / tpl, j = io ? tid / RC : tid % tpl;
        const bool act = io ? tid < RC * tpl : line < RC;
        double2 v[8];
        if (act) {
            double2 *x = X + line * stride;
#pragma unroll
            for (int r = 0; r < 8; ++r) v[r] = first ? load(line, j + r * tpl) : x[pidx(j + r * tpl)];
            if (ns > 1) {
                const int jm = j % ns, f = n / (8 * ns);
#pragma unroll
                for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], wpow<INV>(tws, jm * r * f, n));
            }
            dft8<INV>(v);
        }
        __syncthreads();
        if (act) {
            double2 *x = X + line * stride;
            const int base = (j / ns) * ns * 8 + j % ns;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (last) store(line, base + r * ns, v[r]);
                else x[pidx(base + r * ns)] = v[r];
            }
        }
        __syncthreads();
    }
    if (rf > 1) {
        const int ns = n8, line = tid % RC, j = tid / RC;
        const bool act = tid < RC * tpl;
        double2 v[8];  // rf = 2: four butterflies (u, t); rf = 4: two radix-4 groups
        const double2 *x = X + line * stride;
        if (act) {
            if (rf == 2) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = j + q * tpl;  // butterfly b < ns = n/2
                    v[2 * q] = x[pidx(b)];
                    v[2 * q + 1] = cmul(x[pidx(b + ns)], wpow<INV>(tws, b, n));
                    bfly(v[2 * q], v[2 * q + 1]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int b = j + q * tpl;  // b < ns = n/4
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[4 * q + r] = x[pidx(b + r * ns)];
#pragma unroll
                    for (int r = 1; r < 4; ++r) v[4 * q + r] = cmul(v[4 * q + r], wpow<INV>(tws, b * r, n));
                    dft4<INV>(v + 4 * q);
                }
            }
        }
        __syncthreads();
        if (act) {
            if (rf == 2) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = j + q * tpl;
                    store(line, b, v[2 * q]);
                    store(line, b + ns, v[2 * q + 1]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) store(line, j + q * tpl + r * ns, v[4 * q + r]);
            }
        }
        __syncthreads();
    }
}

// One length-n transform along y (axis 1) or z (axis 2) per (line, RHS) of the
// workgroup's line and RHS chunk, on the half spectrum (x extent nh = n/2 + 1);
// the z pass of the centre mode multiplies by a(k) between its forward and inverse
// transforms (the forward transform's last stage writes the products to LDS, where
// the inverse transform's first stage reads them).
__global__ void __launch_bounds__(256) k_fft_axis(const FftPass a) {
    extern __shared__ double2 X[];  // [RC][n + n/8 + 1], see pidx
    __shared__ double2 tws[64];     // the n/2 twiddles (n <= 128)
    const int n = a.n, nh = n / 2 + 1, half_n = n >> 1, stride = n + (n >> 3) + 1;
    for (int e = threadIdx.x; e < half_n; e += 256) tws[e] = a.tw[e];
    __syncthreads();
    const int RC = a.RB < kRC ? a.RB : kRC;
    const int rc0 = blockIdx.y * RC;
    const int L = blockIdx.x, i = L % nh, q = L / nh;  // line (q, i): q = k (axis 1) or j (axis 2)
    const int64_t g0 = a.axis == 1 ? int64_t(q) * n * nh + i : int64_t(q) * nh + i;
    const int64_t ls = a.axis == 1 ? nh : int64_t(n) * nh;
    auto gload = [&](int r, int t) { return a.cin[(g0 + t * ls) * a.RB + rc0 + r]; };
    const double sc = a.mode == kForward ? 1.0 : 1.0 / n;
    auto gstore = [&](int r, int t, double2 v) {
        a.cout[(g0 + t * ls) * a.RB + rc0 + r] = make_double2(sc * v.x, sc * v.y);
    };
    if (a.mode == kForward) {
        line_fft_io<false>(X, stride, n, RC, tws, gload, gstore);
    } else if (a.mode == kInverse) {
        line_fft_io<true>(X, stride, n, RC, tws, gload, gstore);
    } else {
        // a(k) at (kx, ky, kz) = (i, q, t): line L = q * nh + i of the z-ordered table
        const double *amp = a.amp + int64_t(L) * n;
        auto lstore = [&](int r, int t, double2 v) {
            const double w = amp[t];
            X[r * stride + pidx(t)] = make_double2(w * v.x, w * v.y);
        };
        auto lload = [&](int r, int t) { return X[r * stride + pidx(t)]; };
        line_fft_io<false>(X, stride, n, RC, tws, gload, lstore);
        line_fft_io<true>(X, stride, n, RC, tws, lload, gstore);
    }
}

// The x passes: real lines of n points <-> their n/2 + 1 spectrum values, through one
// complex transform of length m = n/2 of z[p] = x[2p] + i x[2p+1].  With Z = DFT_m(z),
// w = exp(-2 pi i / n) and k = 0..m (Z[m] = Z[0]):
//   X[k] = E[k] + w^k O[k],  E[k] = (Z[k] + conj Z[m-k]) / 2,  O[k] = -i (Z[k] - conj Z[m-k]) / 2,
// and back: Z[k] = E[k] + i O[k] with E[k] = (X[k] + conj X[m-k]) / 2 and
// O[k] = w^-k (X[k] - conj X[m-k]) / 2, z = IDFT_m(Z) / m (the inverse's 1/n included).
__global__ void __launch_bounds__(256) k_fft_x(const FftPass a) {
    extern __shared__ double2 X[];  // [RC][m + m/8 + 1], see pidx
    __shared__ double2 tws[64], twh[32];  // the n/2 twiddles of length n, the m/2 of length m
    const int n = a.n, m = n >> 1, nh = m + 1, stride = m + (m >> 3) + 1;
    for (int e = threadIdx.x; e < m; e += 256) tws[e] = a.tw[e];
    for (int e = threadIdx.x; e < m / 2; e += 256) twh[e] = a.tw[2 * e];
    __syncthreads();
    const int RC = a.RB < kRC ? a.RB : kRC;
    const int rc0 = blockIdx.y * RC;
    const int64_t L = blockIdx.x;  // line (k, j): real points g = L*n + t, spectrum h = L*nh + k
    auto lload = [&](int r, int t) { return X[r * stride + pidx(t)]; };
    auto lstore = [&](int r, int t, double2 v) { X[r * stride + pidx(t)] = v; };
    if (a.mode == kForward) {
        auto rload = [&](int r, int p) {
            const int64_t g = (L * n + 2 * p) * a.RB + rc0 + r;
            return make_double2(a.rin[g], a.rin[g + a.RB]);
        };
        line_fft_io<false>(X, stride, m, RC, twh, rload, lstore);
        for (int e = threadIdx.x; e < nh * RC; e += 256) {
            const int k = e / RC, r = e % RC;
            const double2 zk = X[r * stride + pidx(k % m)], zc = conjg(X[r * stride + pidx((m - k) % m)]);
            const double2 ev = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
            const double2 od = make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x));  // -i (zk - zc) / 2
            a.cout[(L * nh + k) * a.RB + rc0 + r] = cadd(ev, cmul(wpow<false>(tws, k, n), od));
        }
    } else {
        constexpr int kPerX = kPer / 2;  // m * RC / 256 elements per thread at most
        double2 vk[kPerX], vc[kPerX];
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            const int e = threadIdx.x + u * 256, k = e / RC, r = e % RC;
            double2 xk = make_double2(0.0, 0.0), xc = xk;
            if (e < m * RC) {
                xk = a.cin[(L * nh + k) * a.RB + rc0 + r];
                xc = a.cin[(L * nh + m - k) * a.RB + rc0 + r];
            }
            vk[u] = xk;
            vc[u] = xc;
        }
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            const int e = threadIdx.x + u * 256, k = e / RC, r = e % RC;
            if (e < m * RC) {
                const double2 xk = vk[u], xc = conjg(vc[u]);
                const double2 ev = make_double2(0.5 * (xk.x + xc.x), 0.5 * (xk.y + xc.y));
                const double2 od = cmul(wpow<true>(tws, k, n), make_double2(0.5 * (xk.x - xc.x), 0.5 * (xk.y - xc.y)));
                X[r * stride + pidx(k)] = make_double2(ev.x - od.y, ev.y + od.x);  // E + i O
            }
        }
        __syncthreads();
        line_fft_io<true>(X, stride, m, RC, twh, lload, lstore);
        // the real points, two neighbouring RHS per 16-byte access when the chunk is even
        // (RC = 1: one), with the added values loaded before any is used
        const double sc = 1.0 / m;
        const int rw = RC % 2 == 0 ? 2 : 1, nw = m * RC / rw;
        double2 d0[kPerX], d1[kPerX];  // added values at points 2p and 2p + 1 of RHS r (, r + 1)
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            const int e = threadIdx.x + u * 256, p = e / (RC / rw), r = (e % (RC / rw)) * rw;
            const int64_t g = (L * n + 2 * p) * a.RB + rc0 + r;
            double2 x0 = make_double2(0.0, 0.0), x1 = x0;
            if (a.add && e < nw) {
                if (rw == 2) {
                    x0 = *reinterpret_cast<const double2 *>(a.add + g);
                    x1 = *reinterpret_cast<const double2 *>(a.add + g + a.RB);
                } else {
                    x0.x = a.add[g];
                    x1.x = a.add[g + a.RB];
                }
            }
            d0[u] = x0;
            d1[u] = x1;
        }
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            const int e = threadIdx.x + u * 256, p = e / (RC / rw), r = (e % (RC / rw)) * rw;
            if (e < nw) {
                const int64_t g = (L * n + 2 * p) * a.RB + rc0 + r;
                const double2 v = X[r * stride + pidx(p)];  // (point 2p, point 2p + 1) of RHS r
                if (rw == 2) {
                    const double2 w = X[(r + 1) * stride + pidx(p)];
                    *reinterpret_cast<double2 *>(a.rout + g) = make_double2(sc * v.x + d0[u].x, sc * w.x + d0[u].y);
                    *reinterpret_cast<double2 *>(a.rout + g + a.RB) =
                        make_double2(sc * v.y + d1[u].x, sc * w.y + d1[u].y);
                } else {
                    a.rout[g] = sc * v.x + d0[u].x;
                    a.rout[g + a.RB] = sc * v.y + d1[u].x;
                }
            }
        }
    }
}

// out[q][r] = sum_c iw[q][c] u[ig[q][c]][r]  (trilinear, 8 corners per node)
template <typename TO>
__global__ void __launch_bounds__(256) k_interp(const double *u, const int32_t *ig, const double *iw, int64_t N,
                                                int RB, TO *out) {
    const int64_t total = N * RB;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t q = e / RB;
        const int r = int(e % RB);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += iw[q * 8 + c] * u[int64_t(ig[q * 8 + c]) * RB + r];
        out[e] = static_cast<TO>(acc);
    }
}

// g[gi][r] = scale * sum over the nodes interpolating from grid point gi of w * v[q][r]
// (the transpose of k_interp in gather form: CSR by grid point, no atomics)
template <typename TI>
__global__ void __launch_bounds__(256) k_interp_t(const TI *v, const int32_t *tptr, const int32_t *tq,
                                                  const double *tw, int64_t G, int RB, double scale, double *g) {
    const int64_t total = G * RB;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        const int64_t gi = e / RB;
        const int r = int(e % RB);
        double acc = 0.0;
        for (int k = tptr[gi]; k < tptr[gi + 1]; ++k) acc += tw[k] * static_cast<double>(v[int64_t(tq[k]) * RB + r]);
        g[e] = scale * acc;
    }
}

int grid_of(int64_t total) {
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    return int(g < 65536 ? g : 65536);
}

void fft_pass(const SpecOps &sp, int RB, int axis, int mode, const double *rin, const double *cin, double *cout,
              double *rout, const double *add, hipStream_t s) {
    FftPass a;
    a.rin = rin;
    a.cin = reinterpret_cast<const double2 *>(cin);
    a.cout = reinterpret_cast<double2 *>(cout);
    a.rout = rout;
    a.add = add;
    a.amp = sp.amp;
    a.tw = reinterpret_cast<const double2 *>(sp.tw);
    a.n = sp.n;
    a.RB = RB;
    a.axis = axis;
    a.mode = mode;
    const int RC = RB < kRC ? RB : kRC;
    const unsigned n = unsigned(sp.n), nh = n / 2 + 1;
    if (axis == 0) {
        const size_t lds = size_t(n / 2 + n / 16 + 1) * RC * sizeof(double2);
        hipLaunchKernelGGL(k_fft_x, dim3(n * n, unsigned(RB / RC)), dim3(256), lds, s, a);
    } else {
        const size_t lds = size_t(n + n / 8 + 1) * RC * sizeof(double2);
        hipLaunchKernelGGL(k_fft_axis, dim3(n * nh, unsigned(RB / RC)), dim3(256), lds, s, a);
    }
}

// g (real [G][RB]) -> filtered real field, written to rout (+ add); gc holds the half spectrum
void filter(const SpecOps &sp, int RB, const double *g, double *gc, double *rout, const double *add, hipStream_t s) {
    fft_pass(sp, RB, 0, kForward, g, nullptr, gc, nullptr, nullptr, s);
    fft_pass(sp, RB, 1, kForward, nullptr, gc, gc, nullptr, nullptr, s);
    fft_pass(sp, RB, 2, kCentre, nullptr, gc, gc, nullptr, nullptr, s);
    fft_pass(sp, RB, 1, kInverse, nullptr, gc, gc, nullptr, nullptr, s);
    fft_pass(sp, RB, 0, kInverse, nullptr, gc, nullptr, rout, add, s);
}

}  // namespace

bool spectral_rb_ok(int RB) { return RB <= kRC || RB % kRC == 0; }

void launch_spectral(const SpecOps &sp, int RB, const double *x, double *gr, double *gc, Prec out_prec, void *y,
                     int64_t N, hipStream_t s) {
    filter(sp, RB, x, gc, gr, nullptr, s);
    if (out_prec == Prec::F64)
        hipLaunchKernelGGL(k_interp<double>, dim3(grid_of(N * RB)), dim3(256), 0, s, gr, sp.ig, sp.iw, N, RB,
                           static_cast<double *>(y));
    else
        hipLaunchKernelGGL(k_interp<float>, dim3(grid_of(N * RB)), dim3(256), 0, s, gr, sp.ig, sp.iw, N, RB,
                           static_cast<float *>(y));
}

void launch_spectral_t(const SpecOps &sp, int RB, const void *v, Prec in_prec, double scale, const double *add,
                       double *gr, double *gc, double *y, hipStream_t s) {
    const int64_t G = sp.G;
    if (in_prec == Prec::F64)
        hipLaunchKernelGGL(k_interp_t<double>, dim3(grid_of(G * RB)), dim3(256), 0, s, static_cast<const double *>(v),
                           sp.tptr, sp.tq, sp.tw8, G, RB, scale, gr);
    else
        hipLaunchKernelGGL(k_interp_t<float>, dim3(grid_of(G * RB)), dim3(256), 0, s, static_cast<const float *>(v),
                           sp.tptr, sp.tq, sp.tw8, G, RB, scale, gr);
    filter(sp, RB, gr, gc, y, add, s);
}

}  // namespace pat
