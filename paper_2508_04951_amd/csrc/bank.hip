// bank.hip -- a bank of Doppler hypotheses on one pulse: y_h[m] = sum_n x[n] h(alpha_h m - n)
// (Eq 2 resampled with the windowed sum of Eq 17) for many alpha_h at once.
//
// Farrow filter bank.  Output m of hypothesis h sits at t = alpha_h m = f + mu (f integer,
// mu in [0, 1)) and takes taps f + j, j = -H + 1 .. H, with weights h(mu - j).  Each weight is
// a polynomial in s = 2 mu - 1: h(mu - j) ~= sum_r d_r[j] s^r (r < R), so
//     y_h[m] = sum_r s^r Z[f][r],   Z[f][r] = sum_j x[f + j] d_r[j].
// Z depends on the input position only: it is computed once per pulse (k_farrow_z, R FIR
// filters of 2H taps) and every hypothesis then costs one Horner sum of R terms per output
// (k_farrow_bank).  The polynomials interpolate h at the R Chebyshev nodes of [0, 1] in
// float64 (k_farrow_coef), in the Chebyshev basis and then converted to powers of s: the
// Chebyshev coefficients of these smooth functions decay fast, so the power basis loses
// little, and Horner costs half the vector work of a Clenshaw sum.  At R = 8 the bank is within
// ~4e-7 rel-L2 of the direct sum at H = 64 and 128.  An output whose position is an exact
// integer takes the input sample.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rc_internal.h"

namespace rc {
namespace {

constexpr int kR = kFarrowOrders;
constexpr int kBankM = 256;        // outputs per workgroup and hypothesis
constexpr int kBankThreads = 256;

__device__ __forceinline__ double kaiser_series(const KaiserPoly &kp, double x)
{
    const double s = 1.0 - x * x;
    double acc = kp.c[kp.n - 1];
    for (int j = kp.n - 2; j >= 0; --j)
        acc = fma(acc, s, kp.c[j]);
    return acc;
}

// coef[(j + H - 1) * R + r] = d_r[j]: the polynomial in s = 2 mu - 1 that interpolates
// mu -> h(mu - j) at the R Chebyshev nodes of [0, 1].  One thread per tap, all in float64: the
// Chebyshev coefficients c_r, then d = sum_r c_r T_r(s) expanded in powers of s.
__global__ void __launch_bounds__(256) k_farrow_coef(KaiserPoly kp, int H, int taper, float *__restrict__ coef)
{
    const int tap = blockIdx.x * 256 + threadIdx.x;
    if (tap >= 2 * H)
        return;
    const int j = tap - H + 1;
    double w[kR];
    for (int i = 0; i < kR; ++i) {
        const double th = (i + 0.5) / kR;            // node angle / pi
        const double mu = 0.5 * (cospi(th) + 1.0);   // in (0, 1): |mu - j| < H for every tap
        const double u = mu - (double)j;
        double v = sinpi(u) / (kPi * u);
        if (taper)
            v *= kaiser_series(kp, u / (double)H);
        w[i] = v;
    }
    // power-basis coefficients of T_r (rows r), by T_{r+1} = 2 s T_r - T_{r-1}
    double T[kR][kR] = {};
    T[0][0] = 1.0;
    if (kR > 1)
        T[1][1] = 1.0;
    for (int r = 1; r + 1 < kR; ++r)
        for (int k = 0; k < kR; ++k)
            T[r + 1][k] = (k > 0 ? 2.0 * T[r][k - 1] : 0.0) - T[r - 1][k];
    double d[kR] = {};
    for (int r = 0; r < kR; ++r) {
        double c = 0.0;
        for (int i = 0; i < kR; ++i)
            c = fma(w[i], cospi(r * ((i + 0.5) / kR)), c);
        c *= (r == 0 ? 1.0 : 2.0) / kR;
        for (int k = 0; k < kR; ++k)
            d[k] = fma(c, T[r][k], d[k]);
    }
    for (int k = 0; k < kR; ++k)
        gmem(coef)[tap * kR + k] = (float)d[k];
}

// Z[f][r] for f in [0, F) on the matrix cores: for 16 consecutive positions p0 + i the filter
// bank is the product of the Hankel matrix A[i][t] = x[p0 + i - H + 1 + t] (16 x 2H) and the
// coefficient matrix C[t][r] (2H x 8).  Three precisions (rc_bank_precision):
//   FP16X3, BF16X3  32 taps per v_mfma_f32_16x16x32_f16 / _bf16.  Both operands are split into
//                   half-precision hi + lo parts after exact power-of-two scaling (the samples by a
//                   workgroup-wide exponent, the coefficients by 2^kZCoefExp).  The B operand holds
//                   C_hi in columns 0..7 and C_lo in columns 8..15, so the two products A_hi B and
//                   A_lo B of one accumulator give A (C_hi + C_lo) once the column halves are added:
//                   A_hi C_hi + A_hi C_lo + A_lo C_hi (+ A_lo C_lo) in float32, about 22 bits per
//                   product with float16 (11-bit significands) and about 16 with bfloat16 (8-bit).
//                   A row i of the Hankel matrix starts at span offset i, which is 16-byte aligned
//                   only for i % 8 == 0, so the span is staged as 8 copies shifted by 0..7 samples
//                   and row i reads copy i % 8 at the aligned offset i - i % 8.
//   FP32            4 taps per v_mfma_f32_16x16x4_f32 on the float32 samples and coefficients
//                   (k_farrow_z_f32), columns 8..15 of B unused.
constexpr int kZPos = 256;                                   // positions per workgroup
constexpr int kZCoefExp = 12;

__host__ __device__ constexpr int farrow_z_steps(int H) { return (2 * H + 31) / 32; }
// staged span (samples) of one workgroup: kZPos + 32 steps, plus 8 for the shifted copies
__host__ __device__ constexpr int farrow_z_span(int H) { return kZPos + 32 * farrow_z_steps(H); }
size_t farrow_z_lds_bytes(int H)
{
    const size_t L = (size_t)farrow_z_span(H);
    return (L + 8) * sizeof(float2) + 8 * 4 * L * sizeof(_Float16) + 16;
}

typedef float zfloatx4 __attribute__((ext_vector_type(4)));

// The half-precision element, its 8-wide MFMA operand and the 16x16x32 product of a precision.
template <int P>
struct ZHalf;
template <>
struct ZHalf<RC_BANK_FP16X3> {
    typedef _Float16 T;
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ zfloatx4 mfma(v8 a, v8 b, zfloatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct ZHalf<RC_BANK_BF16X3> {
    typedef __bf16 T;
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ zfloatx4 mfma(v8 a, v8 b, zfloatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// Persistent: each workgroup builds its B fragments once, then walks blocks of kZPos positions
// (blockIdx.x, + gridDim.x, ...), loading the next block's span into registers while the
// current block's products run.  KS bounds the 32-tap steps (4, 8 or 16: H <= 64, 128, 256),
// which sets the registers the fragments and the prefetch hold; P the half precision.
template <int KS, int P>
__global__ void __launch_bounds__(256) k_farrow_z(const float2 *__restrict__ x, int64_t n, int64_t F, int H,
                                                  const float *__restrict__ coef, float2 *__restrict__ Z)
{
    typedef typename ZHalf<P>::T half_t;
    typedef typename ZHalf<P>::v8 half8;
    constexpr int kZMaxSteps = KS;
    constexpr int kZPrefetch = (kZPos + 32 * KS + 8 + 255) / 256;  // span samples per thread
    extern __shared__ __attribute__((aligned(16))) float2 smem_z[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ksteps = farrow_z_steps(H), L = farrow_z_span(H);
    float2 *stage = smem_z;                                                  // L + 8 samples
    half_t *copies = reinterpret_cast<half_t *>(stage + L + 8);              // [8 shifts][4 planes][L]
    float *wmax = reinterpret_cast<float *>(copies + 8 * 4 * L);             // 4 wave maxima
    const int64_t nblk = (F + kZPos - 1) / kZPos;
    // the span of block b: sample k is x[b kZPos - H + 1 + k], zero outside [0, n)
    float2 pre[kZPrefetch];
    auto fetch = [&](int64_t b) {
        const int64_t g0 = b * kZPos - H + 1;
#pragma unroll
        for (int u = 0; u < kZPrefetch; ++u) {
            const int k = tid + 256 * u;
            const int64_t g = g0 + k;
            pre[u] = (k < L + 8 && g >= 0 && g < n) ? gload(x, g) : make_float2(0.f, 0.f);
        }
    };
    fetch(blockIdx.x);
    // B fragments (this lane's column: order r = col % 8, hi part for col < 8, lo part above),
    // built once while the first span is in flight
    const int col = lane & 15, q = lane >> 4;
    half8 bfrag[kZMaxSteps];
#pragma unroll
    for (int st = 0; st < kZMaxSteps; ++st) {
        if (st < ksteps) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int t = 32 * st + 8 * q + j;
                const float c = t < 2 * H ? ldexpf(gload(coef, (int64_t)t * kR + (col & 7)), kZCoefExp) : 0.f;
                const half_t hi = (half_t)c;
                bfrag[st][j] = col < 8 ? hi : (half_t)(c - (float)hi);
            }
        }
    }
    const int i = col;  // A row (position within a tile) of this lane
    const half_t *cbase = copies + (size_t)(i & 7) * 4 * L + (i & ~7) + 8 * q;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        float m = 0.f;
#pragma unroll
        for (int u = 0; u < kZPrefetch; ++u) {
            const int k = tid + 256 * u;
            if (k < L + 8) {
                stage[k] = pre[u];
                m = fmaxf(m, fmaxf(fabsf(pre[u].x), fabsf(pre[u].y)));
            }
        }
        for (int o = 32; o > 0; o >>= 1)
            m = fmaxf(m, __shfl_xor(m, o, 64));
        if (lane == 0)
            wmax[wave] = m;
        if (b + gridDim.x < nblk)
            fetch(b + gridDim.x);
        __syncthreads();
        int ex = 0;
        (void)frexpf(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])), &ex);
        const int sexp = 14 - ex;  // scaled samples below 2^14 in magnitude
        // the shifted fp16 copies: copy c, plane (re hi, re lo, im hi, im lo), entry k = span[k + c]
        for (int k = tid; k < L; k += 256) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float2 v = stage[k + c];
                const float re = ldexpf(v.x, sexp), im = ldexpf(v.y, sexp);
                const half_t rh = (half_t)re, ih = (half_t)im;
                half_t *cp = copies + (size_t)c * 4 * L + k;
                cp[0] = rh;
                cp[L] = (half_t)(re - (float)rh);
                cp[2 * L] = ih;
                cp[3 * L] = (half_t)(im - (float)ih);
            }
        }
        __syncthreads();
        const float unscale = ldexpf(1.f, -(sexp + kZCoefExp));
        const int64_t f0 = b * kZPos;
#pragma unroll 1
        for (int tile = wave; tile < kZPos / 16; tile += 4) {
            zfloatx4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < kZMaxSteps; ++st) {
                if (st < ksteps) {
                    const int off = 16 * tile + 32 * st;  // a multiple of 8 halves: 16-byte aligned
                    const half8 arh = *reinterpret_cast<const half8 *>(cbase + off);
                    const half8 arl = *reinterpret_cast<const half8 *>(cbase + L + off);
                    const half8 aih = *reinterpret_cast<const half8 *>(cbase + 2 * L + off);
                    const half8 ail = *reinterpret_cast<const half8 *>(cbase + 3 * L + off);
                    acc_re = ZHalf<P>::mfma(arh, bfrag[st], acc_re);
                    acc_im = ZHalf<P>::mfma(aih, bfrag[st], acc_im);
                    acc_re = ZHalf<P>::mfma(arl, bfrag[st], acc_re);
                    acc_im = ZHalf<P>::mfma(ail, bfrag[st], acc_im);
                }
            }
            // lane (col, q) holds rows 4 q + k of column col: add the lo half (col + 8) to the hi half
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float zr = acc_re[k] + __shfl_xor(acc_re[k], 8, 64);
                const float zi = acc_im[k] + __shfl_xor(acc_im[k], 8, 64);
                const int64_t f = f0 + 16 * tile + 4 * q + k;
                if (col < 8 && f < F)
                    gmem(Z)[f * kR + col] = make_float2(zr * unscale, zi * unscale);
            }
        }
        __syncthreads();  // stage, copies and wmax are rewritten for the next block
    }
}

// Z[f][r] in float32 on the matrix cores: per 16-position tile, v_mfma_f32_16x16x4_f32 over 4 taps
// at a time, lane (i, q) = (lane % 16, lane / 16) holding A[i][4 st + q] = x[p0 + i - H + 1 + 4 st + q]
// and B[4 st + q][col] = C[4 st + q][col] (zero for col >= 8).  One workgroup per block of kZPos
// positions: the span and the coefficient matrix are staged in LDS once.
size_t farrow_z_f32_lds_bytes(int H)
{
    return (size_t)(kZPos + 2 * H + 4) * sizeof(float2) + (size_t)(2 * H + 4) * kR * sizeof(float);
}

__global__ void __launch_bounds__(256) k_farrow_z_f32(const float2 *__restrict__ x, int64_t n, int64_t F, int H,
                                                      const float *__restrict__ coef, float2 *__restrict__ Z)
{
    extern __shared__ __attribute__((aligned(16))) float2 smem_z32[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int taps = 2 * H, steps = (taps + 3) / 4;
    const int L = kZPos + 4 * steps;                                          // span samples
    float2 *span = smem_z32;
    float *cl = reinterpret_cast<float *>(span + L);                          // [4 steps][8], zero-padded
    const int64_t f0 = (int64_t)blockIdx.x * kZPos, g0 = f0 - H + 1;
    for (int k = tid; k < L; k += 256) {
        const int64_t g = g0 + k;
        span[k] = (g >= 0 && g < n) ? gload(x, g) : make_float2(0.f, 0.f);
    }
    for (int e = tid; e < 4 * steps * kR; e += 256)
        cl[e] = e < taps * kR ? gload(coef, (int64_t)e) : 0.f;
    __syncthreads();
    const int col = lane & 15, q = lane >> 4, i = col;
#pragma unroll 1
    for (int tile = wave; tile < kZPos / 16; tile += 4) {
        zfloatx4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
        const float2 *arow = span + 16 * tile + i + q;
        const float *bcol = cl + q * kR + (col & 7);
#pragma unroll 4
        for (int st = 0; st < steps; ++st) {
            const float2 a = arow[4 * st];
            const float b = col < 8 ? bcol[4 * st * kR] : 0.f;
            acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b, acc_im, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t f = f0 + 16 * tile + 4 * q + k;
            if (col < 8 && f < F)
                gmem(Z)[f * kR + col] = make_float2(acc_re[k], acc_im[k]);
        }
    }
}

// One group of hypotheses (consecutive in alpha order) for kBankM outputs: the Z rows the
// group touches are staged in LDS, then each thread walks its outputs for every hypothesis.
struct BankGroup {
    int first;  // index into the alpha-sorted list
    int count;
};

__global__ void __launch_bounds__(kBankThreads)
k_farrow_bank(const float2 *__restrict__ Z, int64_t F, const float2 *__restrict__ x, int64_t n,
              const double *__restrict__ alpha, const int *__restrict__ hyp, const BankGroup *__restrict__ groups,
              int64_t n_out, float2 *__restrict__ y, int max_rows)
{
    // LDS: the group's Z rows as R / 2 planes of float4 (plane q holds Z_{2q}, Z_{2q+1} of every
    // row, so the lanes of a wave, whose rows are consecutive, read consecutive 16-byte slots),
    // then the input samples at the same positions (an exact sample instant reads LDS, so no load
    // ever sits between two output stores)
    extern __shared__ __attribute__((aligned(16))) float4 zs[];
    const int tid = threadIdx.x;
    const BankGroup g = gload(groups, blockIdx.y);
    const int64_t m0 = (int64_t)blockIdx.x * kBankM;
    const int64_t mlast = (m0 + kBankM < n_out ? m0 + kBankM : n_out) - 1;
    // alphas are sorted: the group's rows are floor(a_first m0) .. floor(a_last mlast)
    const double alo = gload(alpha, g.first), ahi = gload(alpha, g.first + g.count - 1);
    const int64_t fmin = (int64_t)floor(__dmul_rn(alo, (double)m0));
    const int64_t fmax = (int64_t)floor(__dmul_rn(ahi, (double)mlast));
    const int rows = (int)(fmax - fmin + 1);
    if (rows > max_rows)
        return;  // the host sizes groups so this never happens; uniform over the workgroup
    // staging in rounds of 8 loads per thread, issued before any is waited for; indices are
    // clamped into the buffers and what lies outside them is zeroed
    const auto zg = gmem(reinterpret_cast<const float4 *>(Z));
    const int64_t zlast = F * (kR / 2) - 1;
    for (int e0 = 0; e0 < rows * (kR / 2); e0 += 8 * kBankThreads) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t gi = fmin * (kR / 2) + e0 + u * kBankThreads + tid;
            const float4 t = zg[gi < zlast ? gi : zlast];
            const bool ok = gi <= zlast;
            v[u] = make_float4(ok ? t.x : 0.f, ok ? t.y : 0.f, ok ? t.z : 0.f, ok ? t.w : 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kBankThreads + tid;  // row e / (R / 2), plane e % (R / 2)
            if (e < rows * (kR / 2))
                zs[(e % (kR / 2)) * max_rows + e / (kR / 2)] = v[u];
        }
    }
    float2 *xs = reinterpret_cast<float2 *>(zs + max_rows * (kR / 2));
    const auto xg = gmem(x);
    for (int e0 = 0; e0 < rows; e0 += 8 * kBankThreads) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t f = fmin + e0 + u * kBankThreads + tid;
            const float2 t = xg[f < n ? f : n - 1];
            v[u] = make_float2(f < n ? t.x : 0.f, f < n ? t.y : 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kBankThreads + tid;
            if (e < rows)
                xs[e] = v[u];
        }
    }
    __syncthreads();
    constexpr int Q = kBankM / kBankThreads;
    double md[Q];  // this thread's output indices, as doubles (exact below 2^53)
#pragma unroll
    for (int q = 0; q < Q; ++q)
        md[q] = (double)(m0 + tid + kBankThreads * q);
    const bool full = m0 + kBankM <= n_out;  // uniform: no output of the block past n_out
    const double fmind = (double)fmin;
    for (int i = 0; i < g.count; ++i) {
        const double a = gload(alpha, g.first + i);
        float2 *yh = y + (int64_t)gload(hyp, g.first + i) * n_out + m0 + tid;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (!full && m0 + tid + kBankThreads * q >= n_out)
                continue;
            const double t = __dmul_rn(a, md[q]);
            const double fd = floor(t);
            float2 out;
            if (t == fd) {  // exact sample instant: the input sample itself
                out = xs[(int)(fd - fmind)];
            } else {
                // Horner in s = 2 mu - 1
                const float s = fmaf(2.f, (float)(t - fd), -1.f);
                const float4 *row = zs + (int)(fd - fmind);
                float zr[kR], zi[kR];
#pragma unroll
                for (int q2 = 0; q2 < kR / 2; ++q2) {
                    const float4 z = row[q2 * max_rows];  // (Z_{2 q2}, Z_{2 q2 + 1})
                    zr[2 * q2] = z.x;
                    zi[2 * q2] = z.y;
                    zr[2 * q2 + 1] = z.z;
                    zi[2 * q2 + 1] = z.w;
                }
                float yr = zr[kR - 1], yi = zi[kR - 1];
#pragma unroll
                for (int r = kR - 2; r >= 0; --r) {
                    yr = fmaf(yr, s, zr[r]);
                    yi = fmaf(yi, s, zi[r]);
                }
                out = make_float2(yr, yi);
            }
            store_nt(yh + kBankThreads * q, out);  // written once, read by no later kernel here
        }
    }
}

}  // namespace

bool farrow_eligible(const rc_sinc &k, const double *alphas, int n_hyp)
{
    if (k.half_width < 1 || k.half_width > kFarrowMaxHalfWidth)
        return false;
    if (k.window != RC_WIN_KAISER && k.window != RC_WIN_RECT)
        return false;
    if (k.window == RC_WIN_KAISER && make_kaiser_poly(k.kaiser_beta).n > 56)
        return false;
    for (int i = 0; i < n_hyp; ++i)
        if (!(alphas[i] > 0.0 && alphas[i] <= kFarrowMaxAlpha))
            return false;
    return true;
}

hipError_t build_farrow_coef(const rc_sinc &k, void **dev, std::vector<void *> &allocs)
{
    const int H = k.half_width;
    const size_t bytes = (size_t)2 * H * kR * sizeof(float);
    hipError_t e = hipMalloc(dev, bytes);
    if (e != hipSuccess)
        return e;
    allocs.push_back(*dev);
    const KaiserPoly kp = make_kaiser_poly(k.window == RC_WIN_KAISER ? k.kaiser_beta : 0.0);
    hipLaunchKernelGGL(k_farrow_coef, dim3((2 * H + 255) / 256), dim3(256), 0, 0, kp, H,
                       k.window == RC_WIN_KAISER ? 1 : 0, static_cast<float *>(*dev));
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return hipStreamSynchronize(0);
}

FarrowPlan plan_farrow_bank(int64_t n, int64_t n_out, int H, const double *alphas, int n_hyp)
{
    FarrowPlan p;
    p.n_hyp = n_hyp;
    std::vector<int> order((size_t)n_hyp);
    for (int i = 0; i < n_hyp; ++i)
        order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return alphas[a] < alphas[b]; });
    p.alpha.resize((size_t)n_hyp);
    p.hyp.resize((size_t)n_hyp);
    double amax = 0.0;
    for (int i = 0; i < n_hyp; ++i) {
        p.hyp[(size_t)i] = order[(size_t)i];
        p.alpha[(size_t)i] = alphas[order[(size_t)i]];
        amax = std::max(amax, p.alpha[(size_t)i]);
    }
    // groups: at most 256 hypotheses whose positions at the last output spread by <= 192 samples
    // (one staging of the Z rows then serves every hypothesis of a dense bank)
    const double last = (double)(n_out - 1);
    for (int s = 0; s < n_hyp;) {
        int e = s + 1;
        while (e < n_hyp && e - s < 256 && (p.alpha[(size_t)e] - p.alpha[(size_t)s]) * last <= 192.0)
            ++e;
        p.groups.push_back({s, e - s});
        s = e;
    }
    // rows one group touches in a kBankM block: floor(a_hi mlast) - floor(a_lo m0) + 1
    //   <= a_hi (kBankM - 1) + (a_hi - a_lo) m0 + 2
    p.max_rows = (int)std::ceil(amax * (kBankM - 1) + 192.0) + 3;
    p.F = std::min<int64_t>((int64_t)std::floor(amax * last) + 1, n + H);
    if (p.F < 1)
        p.F = 1;
    p.z_bytes = (size_t)p.F * kR * sizeof(float2);
    p.lds_bytes = (size_t)p.max_rows * (kR + 1) * sizeof(float2);  // Z rows, then the samples
    return p;
}

size_t farrow_desc_bytes(const FarrowPlan &p)
{
    return p.alpha.size() * sizeof(double) + p.hyp.size() * sizeof(int) + p.groups.size() * 8;
}

void farrow_pack_desc(const FarrowPlan &p, char *host)
{
    std::memcpy(host, p.alpha.data(), p.alpha.size() * sizeof(double));
    host += p.alpha.size() * sizeof(double);
    std::memcpy(host, p.hyp.data(), p.hyp.size() * sizeof(int));
    host += p.hyp.size() * sizeof(int);
    for (const auto &g : p.groups) {
        const int v[2] = {g.first, g.count};
        std::memcpy(host, v, 8);
        host += 8;
    }
}

hipError_t launch_farrow_bank(const FarrowPlan &p, const float2 *x, int64_t n, float2 *y, int64_t n_out, int H,
                              int precision, const float *coef, const void *desc_dev, void *z_work, hipStream_t s,
                              Profiler *prof)
{
    if (p.lds_bytes > 160 * 1024 || n_out <= 0 || p.groups.empty())
        return hipErrorInvalidValue;
    float2 *Z = static_cast<float2 *>(z_work);
    const char *d = static_cast<const char *>(desc_dev);
    const double *alpha = reinterpret_cast<const double *>(d);
    const int *hyp = reinterpret_cast<const int *>(d + p.alpha.size() * sizeof(double));
    const BankGroup *groups =
        reinterpret_cast<const BankGroup *>(d + p.alpha.size() * sizeof(double) + p.hyp.size() * sizeof(int));
    static bool attr[64] = {false};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    if (!attr[dev]) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_farrow_bank),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess)
            return e;
        attr[dev] = true;
    }
    const size_t zlds = precision == RC_BANK_FP32 ? farrow_z_f32_lds_bytes(H) : farrow_z_lds_bytes(H);
    if (zlds > 64 * 1024)
        return hipErrorInvalidValue;
    if (prof)
        prof->begin(kKFarrowZ, s);
    // persistent workgroups: as many as fit on the device at once, at most one per block
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return e;
    const int64_t zblocks = (p.F + kZPos - 1) / kZPos;
    const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)zlds);
    const int64_t zgrid = std::min<int64_t>(zblocks, (int64_t)std::max(cus, 1) * std::min<int64_t>(per_cu, 4));
    const int ks = farrow_z_steps(H);
    if (zblocks > 0x7fffffff)
        return hipErrorInvalidValue;
    if (precision == RC_BANK_FP32)
        hipLaunchKernelGGL(k_farrow_z_f32, dim3((unsigned)zblocks), dim3(256), zlds, s, x, n, p.F, H, coef, Z);
    else if (precision == RC_BANK_BF16X3 && ks <= 4)
        hipLaunchKernelGGL((k_farrow_z<4, RC_BANK_BF16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    else if (precision == RC_BANK_BF16X3 && ks <= 8)
        hipLaunchKernelGGL((k_farrow_z<8, RC_BANK_BF16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    else if (precision == RC_BANK_BF16X3)
        hipLaunchKernelGGL((k_farrow_z<16, RC_BANK_BF16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    else if (ks <= 4)
        hipLaunchKernelGGL((k_farrow_z<4, RC_BANK_FP16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    else if (ks <= 8)
        hipLaunchKernelGGL((k_farrow_z<8, RC_BANK_FP16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    else
        hipLaunchKernelGGL((k_farrow_z<16, RC_BANK_FP16X3>), dim3((unsigned)zgrid), dim3(256), zlds, s, x, n, p.F, H,
                           coef, Z);
    e = hipGetLastError();
    if (prof)
        prof->end(s);
    if (e != hipSuccess)
        return e;
    const int64_t mblocks = (n_out + kBankM - 1) / kBankM;
    if (mblocks > 0x7fffffff || p.groups.size() > 65535)
        return hipErrorInvalidValue;
    if (prof)
        prof->begin(kKFarrowBank, s);
    hipLaunchKernelGGL(k_farrow_bank, dim3((unsigned)mblocks, (unsigned)p.groups.size()), dim3(kBankThreads),
                       p.lds_bytes, s, Z, p.F, x, n, alpha, hyp, groups, n_out, y, p.max_rows);
    e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace rc
