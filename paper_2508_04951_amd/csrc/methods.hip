// methods.hip -- the paper's other Doppler resampling methods, as baselines beside the
// windowed-sinc path: its own GPU sinc kernels (App. C: Alg. 1 direct, Alg. 3 tiled, Alg. 2
// with a lookup table), linear interpolation and frequency conversion (Sec. I, Table I), and
// FFT P/Q resampling (Sec. I, Sec. III-A).
//
// The sinc kernels keep the paper's structure on purpose (one output per thread in a
// grid-stride loop, the window of 2h + 1 inputs centred on the nearest input, no taper) so the
// App. C ablation can be repeated on this GPU; the production resampler is k_sinc_mfma.
#include "rc_internal.h"

namespace rc {
namespace {

constexpr float kPiF = 3.14159265358979323846f;

// sinc(u) = sin(pi u) / (pi u) per tap, the "calculated sinc value" of Alg. 1 and 3: u is exact
// in float64 (t - n); its nearest integer k is split off exactly, sin(pi u) = (-1)^k sin(pi r)
// with |r| <= 1/2 in float32, and the quotient in float32.  Exact sample instants give exactly
// 1 (u = 0) and 0 (u a nonzero integer, r = 0).
__device__ __forceinline__ float sinc_tap(double u)
{
    if (u == 0.0)
        return 1.f;
    const double k = rint(u);
    float s = sinpif((float)(u - k));
    if ((int64_t)k & 1)
        s = -s;
    return s / (kPiF * (float)u);
}

__device__ __forceinline__ int64_t nearest_input(double t)
{
    return (int64_t)floor(t + 0.5);
}

// Alg. 1: one thread per output in a grid-stride loop, inputs read from global memory.
__global__ void __launch_bounds__(256) k_paper_direct(PaperArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < a.n_out; m += stride) {
        const double t = __dmul_rn(a.alpha, (double)m);
        const int64_t c = nearest_input(t);
        const int64_t lo = c - a.h < 0 ? 0 : c - a.h;
        const int64_t hi = c + a.h > a.n_in - 1 ? a.n_in - 1 : c + a.h;
        float re = 0.f, im = 0.f;
        for (int64_t n = lo; n <= hi; ++n) {
            const float w = sinc_tap(t - (double)n);
            const float2 v = gload(a.x, n);
            re = fmaf(v.x, w, re);
            im = fmaf(v.y, w, im);
        }
        gmem(a.y)[m] = make_float2(re, im);
    }
}

// Alg. 3 ("tiling"): each block stages the inputs its 256 outputs touch in LDS, then every
// thread sums its window from LDS.  The span of a tile is at most ceil(255 alpha) + 2h + 3
// samples (checked on the host against the dynamic LDS size); samples outside [0, n_in) are 0.
__global__ void __launch_bounds__(256) k_paper_tiled(PaperArgs a)
{
    extern __shared__ float2 xs[];
    for (int64_t m0 = (int64_t)blockIdx.x * 256; m0 < a.n_out; m0 += (int64_t)gridDim.x * 256) {
        const int64_t m1 = (m0 + 255 < a.n_out - 1) ? m0 + 255 : a.n_out - 1;
        const int64_t lo = nearest_input(__dmul_rn(a.alpha, (double)m0)) - a.h;
        const int64_t hi = nearest_input(__dmul_rn(a.alpha, (double)m1)) + a.h;
        const int span = (int)(hi - lo + 1);
        __syncthreads();  // the previous tile's reads of xs are done
        for (int i = threadIdx.x; i < span; i += 256) {
            const int64_t n = lo + i;
            xs[i] = (n >= 0 && n < a.n_in) ? gload(a.x, n) : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const int64_t m = m0 + threadIdx.x;
        if (m < a.n_out) {
            const double t = __dmul_rn(a.alpha, (double)m);
            const int64_t c = nearest_input(t);
            // the same taps, in the same order, as k_paper_direct (zeros outside the record)
            const int64_t nlo = c - a.h < 0 ? 0 : c - a.h;
            const int64_t nhi = c + a.h > a.n_in - 1 ? a.n_in - 1 : c + a.h;
            float re = 0.f, im = 0.f;
            for (int64_t n = nlo; n <= nhi; ++n) {
                const float w = sinc_tap(t - (double)n);
                const float2 v = xs[n - lo];
                re = fmaf(v.x, w, re);
                im = fmaf(v.y, w, im);
            }
            gmem(a.y)[m] = make_float2(re, im);
        }
    }
}

// Alg. 2: each block first fills an LDS table with the positive half of sinc, lut[i] =
// sinc(i dx) (float64, rounded once), dx = (h + 1/2) / (lut_size - 1); a tap at distance
// u = |t - n| takes the nearest entry, floor(u / dx + 1/2), in float64 with explicit
// roundings (no contraction), so the index is the same as any IEEE float64 evaluation's.
__global__ void __launch_bounds__(256) k_paper_lut(PaperArgs a)
{
    extern __shared__ float lut[];
    for (int i = threadIdx.x; i < a.lut_size; i += 256) {
        const double xv = __dmul_rn((double)i, a.dx);
        lut[i] = i == 0 ? 1.f : (float)(sinpi(xv) / (kPi * xv));
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < a.n_out; m += stride) {
        const double t = __dmul_rn(a.alpha, (double)m);
        const int64_t c = nearest_input(t);
        const int64_t lo = c - a.h < 0 ? 0 : c - a.h;
        const int64_t hi = c + a.h > a.n_in - 1 ? a.n_in - 1 : c + a.h;
        float re = 0.f, im = 0.f;
        for (int64_t n = lo; n <= hi; ++n) {
            const double u = fabs(t - (double)n);
            const int64_t idx = (int64_t)floor(__dadd_rn(__dmul_rn(u, a.inv_dx), 0.5));
            const float w = idx < a.lut_size ? lut[idx] : 0.f;
            const float2 v = gload(a.x, n);
            re = fmaf(v.x, w, re);
            im = fmaf(v.y, w, im);
        }
        gmem(a.y)[m] = make_float2(re, im);
    }
}

// Linear interpolation at t = alpha m: (1 - mu) x[f] + mu x[f + 1], x = 0 outside [0, n_in).
__global__ void __launch_bounds__(256) k_linear(const float2 *x, int64_t n_in, float2 *y, int64_t n_out,
                                                double alpha)
{
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= n_out)
        return;
    const double t = __dmul_rn(alpha, (double)m);
    const double f = floor(t);
    const float mu = (float)(t - f);
    const int64_t k = (int64_t)f;
    const float2 z = make_float2(0.f, 0.f);
    const float2 p = (k >= 0 && k < n_in) ? gload(x, k) : z;
    const float2 q = (k + 1 >= 0 && k + 1 < n_in) ? gload(x, k + 1) : z;
    gmem(y)[m] = make_float2(fmaf(mu, q.x - p.x, p.x), fmaf(mu, q.y - p.y, p.y));
}

// exp(2 pi i nu m): the cycle count nu m in float64 with whole cycles dropped exactly, the
// remaining fraction in [-1/2, 1/2) to float32 sincospi.
__device__ __forceinline__ float2 turn(double nu, int64_t m)
{
    double cyc = __dmul_rn(nu, (double)m);
    cyc -= floor(cyc);
    if (cyc >= 0.5)
        cyc -= 1.0;
    float s, c;
    sincospif(2.f * (float)cyc, &s, &c);
    return make_float2(c, s);
}

__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Frequency conversion: y[m] = x[m] exp(2 pi i nu m), nu = (alpha - 1) f_ref / fs cycles per
// sample.  y may equal x.
__global__ void __launch_bounds__(256) k_tone(const float2 *x, float2 *y, int64_t n, double nu)
{
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= n)
        return;
    gmem(y)[m] = cmulf(gload(x, m), turn(nu, m));
}

// P/Q: the input spectrum X (n_in bins, natural order) to the conjugate of the output spectrum
// Y (n_out bins): signed bins |k| <= (K - 1) / 2 copied, K = min(n_in, n_out); for even K the
// bin K/2 folds the input bins +K/2 and -K/2 when bins are removed, or takes half the input
// Nyquist bin at +K/2 and at -K/2 when bins are added.  The conjugate feeds the inverse
// transform, done as a forward one: IDFT(Y) = conj(DFT(conj(Y))) / n_out.
__global__ void __launch_bounds__(256) k_pq_resize(const float2 *X, int64_t n_in, float2 *Yc, int64_t n_out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_out)
        return;
    const int64_t K = n_in < n_out ? n_in : n_out, half = (K - 1) / 2;
    float2 v = make_float2(0.f, 0.f);
    if (j <= half) {
        v = gload(X, j);
    } else if (j >= n_out - half) {
        v = gload(X, n_in - (n_out - j));
    } else if ((K & 1) == 0 && (j == K / 2 || j == n_out - K / 2)) {
        if (n_out < n_in) {
            const float2 a = gload(X, K / 2), b = gload(X, n_in - K / 2);
            v = make_float2(a.x + b.x, a.y + b.y);
        } else if (n_out > n_in) {
            const float2 a = gload(X, K / 2);
            v = make_float2(0.5f * a.x, 0.5f * a.y);
        } else {
            v = gload(X, j);
        }
    }
    gmem(Yc)[j] = make_float2(v.x, -v.y);
}

// P/Q output: y[m] = conj(Z[m]) / n_in for m < n_i (Z = DFT(conj(Y))), 0 beyond, optionally
// turned by the frequency conversion of the remaining dilation.  With Z null (no bins to remove
// or add) the record itself is the P/Q result: y[m] = x[m].
__global__ void __launch_bounds__(256) k_pq_post(const float2 *Z, const float2 *x, int64_t ni, float2 *y,
                                                 int64_t n_out, float scale, int tone, double nu)
{
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= n_out)
        return;
    float2 v = make_float2(0.f, 0.f);
    if (m < ni) {
        if (Z) {
            const float2 z = gload(Z, m);
            v = make_float2(z.x * scale, -z.y * scale);
        } else {
            v = gload(x, m);
        }
        if (tone)
            v = cmulf(v, turn(nu, m));
    }
    gmem(y)[m] = v;
}

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

size_t paper_tiled_lds_bytes(double alpha, int h)
{
    return (size_t)(std::ceil(255.0 * alpha) + 2.0 * h + 3.0) * sizeof(float2);
}

hipError_t launch_paper_sinc(const PaperArgs &a, int variant, int blocks, hipStream_t s, Profiler *prof)
{
    if (a.n_out <= 0)
        return hipSuccess;
    int64_t nblk = blocks > 0 ? blocks : (a.n_out + 255) / 256;
    if (nblk > 0x7fffffff)
        nblk = 0x7fffffff;
    if (prof)
        prof->begin(kKPaperSinc, s);
    switch (variant) {
    case RC_PAPER_TILED:
        hipLaunchKernelGGL(k_paper_tiled, dim3((unsigned)nblk), dim3(256), paper_tiled_lds_bytes(a.alpha, a.h), s, a);
        break;
    case RC_PAPER_LUT:
        hipLaunchKernelGGL(k_paper_lut, dim3((unsigned)nblk), dim3(256), (size_t)a.lut_size * sizeof(float), s, a);
        break;
    default:
        hipLaunchKernelGGL(k_paper_direct, dim3((unsigned)nblk), dim3(256), 0, s, a);
    }
    const hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

hipError_t launch_linear(const float2 *x, int64_t n_in, float2 *y, int64_t n_out, double alpha, hipStream_t s,
                         Profiler *prof)
{
    if (n_out <= 0)
        return hipSuccess;
    if (prof)
        prof->begin(kKLinear, s);
    hipLaunchKernelGGL(k_linear, grid_for(n_out), dim3(256), 0, s, x, n_in, y, n_out, alpha);
    const hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

hipError_t launch_tone(const float2 *x, float2 *y, int64_t n, double nu, hipStream_t s, Profiler *prof)
{
    if (n <= 0)
        return hipSuccess;
    if (prof)
        prof->begin(kKTone, s);
    hipLaunchKernelGGL(k_tone, grid_for(n), dim3(256), 0, s, x, y, n, nu);
    const hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

hipError_t launch_pq(const PqArgs &a, const FftPlan &plan_in, const FftPlan &plan_out, const float2 *tw4096,
                     hipStream_t s, Profiler *prof)
{
    hipError_t e = hipSuccess;
    const float2 *Z = nullptr;
    if (a.ni != a.n_in) {
        // X = DFT_n_in(x), natural order
        const BluesteinJob fx{a.x, a.X, a.work, a.n_in, PhaseNum{}, 0.0, 0.0, nullptr};
        e = launch_bluestein_forward(plan_in, tw4096, fx, s, prof);
        if (e != hipSuccess)
            return e;
        if (prof)
            prof->begin(kKPq, s);
        hipLaunchKernelGGL(k_pq_resize, grid_for(a.ni), dim3(256), 0, s, (const float2 *)a.X, a.n_in, a.Y, a.ni);
        e = hipGetLastError();
        if (prof)
            prof->end(s);
        if (e != hipSuccess)
            return e;
        // Z = DFT_ni(conj(Y)), in place
        const BluesteinJob fy{a.Y, a.Y, a.work, a.ni, PhaseNum{}, 0.0, 0.0, nullptr};
        e = launch_bluestein_forward(plan_out, tw4096, fy, s, prof);
        if (e != hipSuccess)
            return e;
        Z = a.Y;
    }
    if (prof)
        prof->begin(kKPq, s);
    hipLaunchKernelGGL(k_pq_post, grid_for(a.n_out), dim3(256), 0, s, Z, a.x, a.ni, a.y, a.n_out,
                       (float)(1.0 / (double)a.n_in), a.tone, a.nu);
    e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace rc
