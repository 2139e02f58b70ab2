// sinc.hip -- Doppler resampling kernels for gfx950: y[m] = sum_n x[n] h(alpha m - n),
// the windowed Whittaker-Shannon sum of Eq (17) evaluated at the dilated instants of Eq (2).
//
// Two kernels:
//  * k_sinc_fast  -- Kaiser taper, |alpha - 1| <= 1e-4 (range rates up to ~15 km/s).
//    Write t = alpha m = m + S + sigma_m with S an integer fixed per 256-output wave tile and
//    sigma_m = sigma_c + delta_m, |delta_m| <= |alpha-1| * 127.5.  Every output of the tile
//    then uses the same 2H+1 inputs relative to m + S, and the tap weight h(sigma_m - k) is
//    replaced by the quadratic in delta_m through three float64 samples of h at Chebyshev
//    nodes of the tile's drift range.  The three coefficients per tap are wave-uniform
//    (broadcast LDS reads); per tap and output the work is 2 FMAs for the weight and 2 for
//    the complex MAC.  The input span of a 1024-output workgroup is staged once in LDS.
//    An output whose position is an exact integer returns that input sample.
//  * k_sinc_direct -- any taper, any alpha > 0, and the full (H = 0) sum: float64 position and
//    sin(pi mu), float32 tap weights (one reciprocal per tap) and accumulation, 1..64 lanes per
//    output with a shuffle reduction.
#include <cmath>

#include "rc_internal.h"

namespace rc {

KaiserPoly make_kaiser_poly(double beta)
{
    KaiserPoly kp{};
    const double q = 0.25 * beta * beta;
    double t = 1.0, sum = 1.0;
    double terms[56];
    terms[0] = 1.0;
    int n = 1;
    for (int j = 1; j < 56; ++j) {
        t *= q / ((double)j * (double)j);
        terms[j] = t;
        sum += t;
        n = j + 1;
        if (t < 1e-18 * sum)
            break;
    }
    kp.n = n;
    for (int j = 0; j < n; ++j) {
        kp.c[j] = terms[j] / sum;
        kp.cf[j] = (float)kp.c[j];
    }
    // the float32 series stops where the remaining terms (all positive, s <= 1) sum below 2^-27
    double tail = 0.0;
    kp.nf = n;
    for (int j = n - 1; j > 0; --j) {
        tail += kp.c[j];
        if (tail >= std::ldexp(1.0, -27))
            break;
        kp.nf = j;
    }
    return kp;
}

bool sinc_fast_eligible(double alpha, const rc_sinc &k)
{
    return k.window == RC_WIN_KAISER && k.half_width >= 1 && k.half_width <= 256 &&
           std::fabs(alpha - 1.0) <= kSincFastMaxEps;
}

namespace {

// The taper in float32 (the direct sum's per-tap weight): s = 1 - x^2 by one fused operation,
// then the series' first nf terms; relative error a few float32 ulp.
__device__ __forceinline__ float kaiser_at_f(const KaiserPoly &kp, float x)
{
    const float s = fmaf(-x, x, 1.0f);
    float acc = kp.cf[kp.nf - 1];
    for (int j = kp.nf - 2; j >= 0; --j)
        acc = fmaf(acc, s, kp.cf[j]);
    return acc;
}

__device__ __forceinline__ double kaiser_at(const KaiserPoly &kp, double x)
{
    const double s = 1.0 - x * x;
    double acc = kp.c[kp.n - 1];
    for (int j = kp.n - 2; j >= 0; --j)
        acc = fma(acc, s, kp.c[j]);
    return acc;
}

// LDS index with one pad slot per 4 samples: lanes reading samples 4 apart hit distinct banks.
__device__ __forceinline__ int xpad(int e) { return e + (e >> 2); }

__host__ __device__ inline int sinc_span(int H, int dshift)
{
    return kSincWgOut + 2 * H + dshift + 9;
}

__host__ __device__ inline int sinc_xs_floats2(int span)
{
    // padded sample slots, rounded up to a float4 boundary
    return ((span + (span >> 2) + 1) + 1) & ~1;
}

__device__ __forceinline__ void mac4(const float4 cf, const float dl[4], float ar[4], float ai[4],
                                     float2 a, float2 b, float2 c, float2 d)
{
    const float2 xv[4] = {a, b, c, d};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float w = fmaf(dl[i], fmaf(dl[i], cf.z, cf.y), cf.x);
        ar[i] = fmaf(xv[i].x, w, ar[i]);
        ai[i] = fmaf(xv[i].y, w, ai[i]);
    }
}

__global__ void __launch_bounds__(256)
k_sinc_fast(const SincJob *__restrict__ jobs, SincJob inl, int H, KaiserPoly kp)
{
    extern __shared__ float4 smem[];
    const SincJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int64_t M0 = (int64_t)blockIdx.x * kSincWgOut;
    if (M0 >= jb.n_out)
        return;  // uniform over the workgroup
    const double alpha = jb.alpha;
    const double eps = alpha - 1.0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ntap = 2 * H + 1;
    const int ntapp = (ntap + 3) & ~3;

    // integer shift S of each wave tile (rint of the drift at the tile centre)
    const double S0 = rint(eps * ((double)M0 + 127.5));
    const double S3 = rint(eps * ((double)(M0 + 3 * kSincWaveOut) + 127.5));
    const int dshift = (int)fabs(S3 - S0);
    const int64_t lo = M0 + (int64_t)fmin(S0, S3) - H;
    const int span = sinc_span(H, dshift);
    float2 *xs = reinterpret_cast<float2 *>(smem);
    float4 *coef = smem + sinc_xs_floats2(span) / 2 + wave * ntapp;

    for (int e = tid; e < span; e += 256) {
        const int64_t pos = lo + e;
        float2 v = make_float2(0.f, 0.f);
        if (pos >= 0 && pos < jb.n_in)
            v = gmem(jb.x)[pos];
        xs[xpad(e)] = v;
    }

    const int64_t m0 = M0 + (int64_t)wave * kSincWaveOut;
    const double Sd = rint(eps * ((double)m0 + 127.5));
    const double sc = eps * ((double)m0 + 127.5) - Sd;  // sigma at the tile centre
    double d = fabs(eps) * 127.5 * 0.86602540378443865;  // Chebyshev nodes of [-D, D]
    if (d < 1e-4)
        d = 1e-4;
    const double nodes[3] = {sc - d, sc, sc + d};
    const double snode[3] = {sinpi(sc - d), sinpi(sc), sinpi(sc + d)};
    const double inv_h = 1.0 / (double)H;
    for (int kk = lane; kk < ntapp; kk += 64) {
        float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
        if (kk < ntap) {
            const int k = kk - H;
            double hv[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double u = nodes[i] - (double)k;
                double h = 0.0;
                if (fabs(u) < (double)H) {
                    // sinc(u) = sin(pi (sigma - k)) / (pi u) = (-1)^k sin(pi sigma) / (pi u)
                    const double sn = (u == 0.0) ? 1.0 : ((k & 1) ? -snode[i] : snode[i]) / (kPi * u);
                    h = sn * kaiser_at(kp, u * inv_h);
                }
                hv[i] = h;
            }
            const double b = (hv[2] - hv[0]) / (2.0 * d);
            const double c = (hv[2] - 2.0 * hv[1] + hv[0]) / (2.0 * d * d);
            cf = make_float4((float)hv[1], (float)b, (float)c, 0.f);
        }
        coef[kk] = cf;
    }
    __syncthreads();
    if (m0 >= jb.n_out)
        return;  // no barrier follows

    const int64_t mb = m0 + (int64_t)kSincLanesOut * lane;
    float dl[4];
    bool exact[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double m = (double)(mb + i);
        // t = alpha m rounded once (no FMA contraction), as the float64 definition does;
        // t - m is exact by Sterbenz's lemma, and so is the integer shift.
        const double sig = (__dmul_rn(alpha, m) - m) - Sd;
        dl[i] = (float)(sig - sc);
        exact[i] = (sig == 0.0);
    }
    const int e0 = (int)(mb + (int64_t)Sd - H - lo);
    float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
    float2 w0 = xs[xpad(e0)], w1 = xs[xpad(e0 + 1)], w2 = xs[xpad(e0 + 2)];
    for (int kk = 0; kk < ntapp; kk += 4) {
        const float2 w3 = xs[xpad(e0 + kk + 3)];
        const float2 w4 = xs[xpad(e0 + kk + 4)];
        const float2 w5 = xs[xpad(e0 + kk + 5)];
        const float2 w6 = xs[xpad(e0 + kk + 6)];
        mac4(coef[kk], dl, ar, ai, w0, w1, w2, w3);
        mac4(coef[kk + 1], dl, ar, ai, w1, w2, w3, w4);
        mac4(coef[kk + 2], dl, ar, ai, w2, w3, w4, w5);
        mac4(coef[kk + 3], dl, ar, ai, w3, w4, w5, w6);
        w0 = w4;
        w1 = w5;
        w2 = w6;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t m = mb + i;
        if (m < jb.n_out) {
            float2 r = make_float2(ar[i], ai[i]);
            if (exact[i])
                r = xs[xpad(e0 + i + H)];
            gmem(jb.y)[m] = r;
        }
    }
}

__global__ void __launch_bounds__(256)
k_sinc_direct(const SincJob *__restrict__ jobs, SincJob inl, int H, int window, KaiserPoly kp,
              int log2g)
{
    const SincJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int G = 1 << log2g;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t m = gid >> log2g;
    const int sub = (int)(gid & (G - 1));
    int mode = 0;  // 0 idle, 1 exact sample, 2 weighted sum
    float re = 0.f, im = 0.f;
    if (m < jb.n_out) {
        const double t = __dmul_rn(jb.alpha, (double)m);
        const double f = floor(t);
        if (t == f) {
            mode = 1;  // only lane 0 of the group carries the sample into the reduction
            if (sub == 0 && f < (double)jb.n_in) {
                const float2 v = gmem(jb.x)[(int64_t)f];
                re = v.x;
                im = v.y;
            }
        } else {
            mode = 2;
            const int64_t fi = (int64_t)f;
            int64_t lo, hi;
            if (H == 0) {
                lo = 0;
                hi = jb.n_in - 1;
            } else if (window == RC_WIN_PAPER) {
                const int64_t c = (int64_t)floor(t + 0.5);
                lo = c - H;
                hi = c + H;
            } else {
                lo = fi - H + 1;
                hi = fi + H;
            }
            if (lo < 0)
                lo = 0;
            if (hi > jb.n_in - 1)
                hi = jb.n_in - 1;
            // sinc(u) = (-1)^(n - fi) sin(pi mu) / (pi u), mu = t - fi: the common factor
            // sin(pi mu) / pi in float64 once, then per tap u = t - n (float64, rounded once to
            // float32: relative error 2^-24 whatever its size) and its float32 reciprocal
            const float spf = (float)(sinpi(t - f) * (1.0 / kPi));
            const bool taper = (H > 0 && window == RC_WIN_KAISER);
            const double inv_h = H > 0 ? 1.0 / (double)H : 0.0;
            for (int64_t n = lo + sub; n <= hi; n += G) {
                const double ud = t - (double)n;
                float w = __builtin_amdgcn_rcpf((float)ud);
                if ((n - fi) & 1)
                    w = -w;
                if (taper)
                    w *= kaiser_at_f(kp, (float)(ud * inv_h));
                const float2 v = gmem(jb.x)[n];
                re = fmaf(v.x, w, re);
                im = fmaf(v.y, w, im);
            }
            re *= spf;
            im *= spf;
        }
    }
    for (int o = G >> 1; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    if (mode != 0 && sub == 0)
        gmem(jb.y)[m] = make_float2(re, im);
}

}  // namespace

size_t sinc_fast_lds_bytes(int half_width)
{
    const int span = sinc_span(half_width, 2);
    const int ntapp = (2 * half_width + 1 + 3) & ~3;
    return (size_t)sinc_xs_floats2(span) * sizeof(float2) + (size_t)4 * ntapp * sizeof(float4);
}

hipError_t launch_sinc_fast(const SincJob *jobs_dev, const SincJob *job_inline, int njobs,
                            int64_t max_out, int half_width, const KaiserPoly &kp, hipStream_t s,
                            Profiler *prof)
{
    if (njobs <= 0 || max_out <= 0)
        return hipSuccess;
    const int64_t nblk = (max_out + kSincWgOut - 1) / kSincWgOut;
    if (nblk > 0x7fffffff || njobs > 65535)
        return hipErrorInvalidValue;
    const SincJob inl = job_inline ? *job_inline : SincJob{};
    const size_t lds = sinc_fast_lds_bytes(half_width);
    if (prof)
        prof->begin(kKSincFast, s);
    hipLaunchKernelGGL(k_sinc_fast, dim3((unsigned)nblk, (unsigned)njobs), dim3(256), lds, s,
                       jobs_dev, inl, half_width, kp);
    const hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

hipError_t launch_sinc_direct(const SincJob *jobs_dev, const SincJob *job_inline, int njobs,
                              int64_t max_out, const rc_sinc &k, const KaiserPoly &kp,
                              int64_t max_taps, hipStream_t s, Profiler *prof)
{
    if (njobs <= 0 || max_out <= 0)
        return hipSuccess;
    int log2g = 0;  // lanes per output: about 32 taps per lane, at most a wave
    while (log2g < 6 && ((int64_t)32 << log2g) < max_taps)
        ++log2g;
    const int64_t threads = max_out << log2g;
    const int64_t nblk = (threads + 255) / 256;
    if (nblk > 0x7fffffff || njobs > 65535)
        return hipErrorInvalidValue;
    const SincJob inl = job_inline ? *job_inline : SincJob{};
    if (prof)
        prof->begin(kKSincDirect, s);
    hipLaunchKernelGGL(k_sinc_direct, dim3((unsigned)nblk, (unsigned)njobs), dim3(256), 0, s,
                       jobs_dev, inl, (int)k.half_width, (int)k.window, kp, log2g);
    const hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace rc
