// Whittle-Matern Fourier-spectral prior on the GPU (Sec. 4.1 eq. (matern-cov-op);
// the construction of Sec. 6.4): p0 = P w with P = I_h F^* diag(a) F, w a latent
// white-noise grid vector, F the 3D DFT on a periodic n^3 box, a(k) the
// square-root spectrum, I_h trilinear interpolation to the mesh nodes.
//
// Layouts: grid vectors [n^3][RB] with grid index g = (k*n + j)*n + i (x fastest)
// and the RHS fastest; complex grid vectors interleave (re, im) per element.
//
// The 3D transform is five launches of one kernel, each a batch of length-n
// radix-2 FFTs along one axis staged in LDS (one line and a chunk of up to 16
// right-hand sides per workgroup): forward x, forward y, then forward z, the
// multiplication by a(k) and the inverse z in the same pass, then inverse y and
// inverse x.  Forward transforms are decimation in time on bit-reversed input
// (natural-order output); inverse ones are decimation in frequency (natural
// input, bit-reversed output), so no separate reordering pass is needed.
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

__device__ __forceinline__ int bitrev(int t, int logn) { return int(__brev(unsigned(t)) >> (32 - logn)); }

constexpr int kRC = 16;  // right-hand sides per workgroup

enum : int { kForward = 0, kInverse = 1, kCentre = 2 };

struct FftPass {
    const double *rin;   // real input [G][RB], or null
    const double2 *cin;  // complex input [G][RB], or null
    double2 *cout;       // complex output, or null
    double *rout;        // real output (the real part), or null
    const double *add;   // added to the real output, or null
    const double *amp;   // a(k) [G] for the centre pass
    const double2 *tw;   // tw[j] = exp(-2 pi i j / n), j < n/2
    int n, logn, RB, axis, mode;
};

// One length-n transform per (line, RHS) of the workgroup's line and RHS chunk.
__global__ void __launch_bounds__(256) k_fft_axis(const FftPass a) {
    extern __shared__ double2 X[];  // [RC][n]
    __shared__ double2 tws[64];     // the n/2 twiddles (n <= 128), read by every stage
    const int n = a.n, half_n = n >> 1;
    for (int e = threadIdx.x; e < half_n; e += 256) tws[e] = a.tw[e];
    const int RC = a.RB < kRC ? a.RB : kRC;
    const int rc0 = blockIdx.y * RC;
    const int L = blockIdx.x;
    int64_t g0, ls;
    if (a.axis == 0) {
        g0 = int64_t(L) * n;
        ls = 1;
    } else if (a.axis == 1) {
        g0 = int64_t(L / n) * n * n + L % n;
        ls = n;
    } else {
        g0 = L;
        ls = int64_t(n) * n;
    }
    for (int e = threadIdx.x; e < n * RC; e += 256) {
        const int t = e / RC, r = e % RC;
        const int64_t gi = (g0 + t * ls) * a.RB + rc0 + r;
        const double2 v = a.rin ? make_double2(a.rin[gi], 0.0) : a.cin[gi];
        X[r * n + (a.mode == kInverse ? t : bitrev(t, a.logn))] = v;
    }
    __syncthreads();
    if (a.mode != kInverse) {
        // decimation in time, exp(-2 pi i ...) twiddles
        for (int s = 1; s <= a.logn; ++s) {
            const int m = 1 << s, half = m >> 1, step = n >> s;
            for (int b = threadIdx.x; b < half_n * RC; b += 256) {
                const int r = b / half_n, bi = b % half_n;
                const int pos = bi % half, i1 = (bi / half) * m + pos, i2 = i1 + half;
                double2 *x = X + r * n;
                const double2 t = cmul(tws[pos * step], x[i2]), u = x[i1];
                x[i1] = cadd(u, t);
                x[i2] = csub(u, t);
            }
            __syncthreads();
        }
    }
    if (a.mode == kCentre) {
        for (int e = threadIdx.x; e < n * RC; e += 256) {
            const int r = e / n, t = e % n;
            const double w = a.amp[g0 + t * ls];
            X[r * n + t] = make_double2(w * X[r * n + t].x, w * X[r * n + t].y);
        }
        __syncthreads();
    }
    if (a.mode != kForward) {
        // decimation in frequency, exp(+2 pi i ...) twiddles; bit-reversed output
        for (int s = a.logn; s >= 1; --s) {
            const int m = 1 << s, half = m >> 1, step = n >> s;
            for (int b = threadIdx.x; b < half_n * RC; b += 256) {
                const int r = b / half_n, bi = b % half_n;
                const int pos = bi % half, i1 = (bi / half) * m + pos, i2 = i1 + half;
                double2 *x = X + r * n;
                const double2 u = x[i1], v = x[i2];
                x[i1] = cadd(u, v);
                x[i2] = cmul(csub(u, v), conjg(tws[pos * step]));
            }
            __syncthreads();
        }
    }
    const double sc = a.mode == kForward ? 1.0 : 1.0 / n;
    for (int e = threadIdx.x; e < n * RC; e += 256) {
        const int t = e / RC, r = e % RC;
        const int64_t gi = (g0 + t * ls) * a.RB + rc0 + r;
        const double2 v = X[r * n + (a.mode == kForward ? t : bitrev(t, a.logn))];
        if (a.rout) a.rout[gi] = sc * v.x + (a.add ? a.add[gi] : 0.0);
        else a.cout[gi] = make_double2(sc * v.x, sc * v.y);
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
    a.logn = sp.logn;
    a.RB = RB;
    a.axis = axis;
    a.mode = mode;
    const int RC = RB < kRC ? RB : kRC;
    const size_t lds = size_t(sp.n) * RC * sizeof(double2);
    hipLaunchKernelGGL(k_fft_axis, dim3(unsigned(sp.n) * unsigned(sp.n), unsigned(RB / RC)), dim3(256), lds, s, a);
}

// g (real [G][RB]) -> filtered real field, written to rout (+ add)
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
