// sinc_mfma.hip -- the windowed-sinc tap sum of Eq (17) (Kaiser taper, Sec. III-B) as a
// matrix product on the gfx950 matrix cores.
//
// A 1024-output workgroup tile shares one integer shift S and one drift polynomial: every
// output m of the tile sits at t = alpha m = m + S + sigma_c + D z_m with |z_m| <= 1 and
// D = |alpha - 1| * 511.5, so its weights are h(sigma_c + D z - k) ~= sum_r a_r[k] z^r,
// a cubic in z interpolated in float64 at four Chebyshev nodes (tap error ~1e-7 for
// |alpha - 1| <= 6e-5).  Then
//     y[m] = sum_r z_m^r Z_r[m],   Z_r[m] = sum_k x[m + S + k] a_r[k],  k = -H .. H,
// and for a 256-output wave tile m = m0 + 16 i + u the contraction is a GEMM
//     Z_r[i][u] = sum_kappa X[i][kappa] B_r[kappa][u],
//     X[i][kappa] = x[m0 + 16 i + S - H + kappa]   (Hankel: 8-sample aligned runs per lane),
//     B_r[kappa][u] = a_r[kappa - u - H]           (the column shift u lives in B).
// kappa runs over 2H + 16 taps rounded up to whole 32-wide MFMA steps.  Both operands are split
// into float16 hi + lo parts after exact power-of-two scaling, and each order and component
// accumulates hi*hi + hi*lo + lo*hi in float32 (v_mfma_f32_16x16x32_f16): about 22 bits per
// product.  The cubic in z is applied to the four float32 accumulators per output at the end.
#include <cmath>

#include "rc_internal.h"

namespace rc {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMfOut = 1024;       // outputs per workgroup
constexpr int kMfOrders = 4;       // cubic in the drift
constexpr int kCoefExp = 12;       // coefficients are scaled by 2^12 before the fp16 split

template <int H>
struct MfGeom {
    static constexpr int ntap = 2 * H + 1;
    static constexpr int kext = ((2 * H + 16) + 31) / 32 * 32;
    static constexpr int ksteps = kext / 32;
    static constexpr int span = kMfOut + kext;                 // staged samples
    static constexpr int spt = (span + 255) / 256;            // staged samples per thread
    static constexpr int a_off = 0;                             // 4 fp16 arrays of `span`
    static constexpr int b_off = 4 * span * 2;                  // ksteps x orders x {hi,lo} x 1 KiB
    static constexpr int c_off = b_off + ksteps * kMfOrders * 2 * 1024;  // float a_r[k]
    static constexpr int m_off = c_off + kMfOrders * ntap * 4;          // 4 floats: wave maxima
    static constexpr int bytes = m_off + 16;
};

__device__ __forceinline__ double kaiser_at_m(const KaiserPoly &kp, double x)
{
    const double s = 1.0 - x * x;
    double acc = kp.c[kp.n - 1];
    for (int j = kp.n - 2; j >= 0; --j)
        acc = fma(acc, s, kp.c[j]);
    return acc;
}

template <int H>
__global__ void __launch_bounds__(256)
k_sinc_mfma(const SincJob *__restrict__ jobs, SincJob inl, KaiserPoly kp, MfmaSincConst mc)
{
    using G = MfGeom<H>;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    _Float16 *a_rh = reinterpret_cast<_Float16 *>(smem + G::a_off);
    _Float16 *a_rl = a_rh + G::span;
    _Float16 *a_ih = a_rl + G::span;
    _Float16 *a_il = a_ih + G::span;
    unsigned char *bsm = smem + G::b_off;
    float *coef = reinterpret_cast<float *>(smem + G::c_off);
    float *wmax = reinterpret_cast<float *>(smem + G::m_off);

    const SincJob jb = jobs ? jobs[blockIdx.y] : inl;
    const int64_t M0 = (int64_t)blockIdx.x * kMfOut;
    if (M0 >= jb.n_out)
        return;  // uniform over the workgroup
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double alpha = jb.alpha, eps = alpha - 1.0;
    const double mcen = (double)M0 + 511.5;
    const double Sd = rint(eps * mcen);
    const int64_t S = (int64_t)Sd;
    const double sc = eps * mcen - Sd;         // sigma at the tile centre
    double D = fabs(eps) * 511.5;
    if (D < 1e-6)
        D = 1e-6;
    const int64_t lo = M0 + S - H;             // first staged sample

    // 1) stage the input span, find its largest component for the power-of-two scaling
    float2 xv[G::spt];
    float mx = 0.f;
#pragma unroll
    for (int q = 0; q < G::spt; ++q) {
        const int e = tid + 256 * q;
        const int64_t pos = lo + e;
        float2 v = make_float2(0.f, 0.f);
        if (e < G::span && pos >= 0 && pos < jb.n_in)
            v = jb.x[pos];
        xv[q] = v;
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    for (int o = 32; o > 0; o >>= 1)
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0)
        wmax[wave] = mx;

    // 2) drift polynomial a_r[k] of every tap (float64 at 4 Chebyshev nodes, then V^-1)
    {
        double sn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            sn[i] = sinpi(sc + D * mc.node[i]);
        const double inv_h = 1.0 / (double)H;
        const float cscale = ldexpf(1.0f, kCoefExp);
        for (int t = tid; t < G::ntap; t += 256) {
            const int k = t - H;
            double hv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double u = (sc + D * mc.node[i]) - (double)k;
                double h = 0.0;
                if (fabs(u) < (double)H) {
                    const double s = (k & 1) ? -sn[i] : sn[i];
                    h = (u == 0.0 ? 1.0 : s / (kPi * u)) * kaiser_at_m(kp, u * inv_h);
                }
                hv[i] = h;
            }
#pragma unroll
            for (int r = 0; r < kMfOrders; ++r) {
                double a = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    a = fma(mc.vinv[r * 4 + i], hv[i], a);
                coef[r * G::ntap + t] = (float)a * cscale;
            }
        }
    }
    __syncthreads();

    // 3) scale and split the staged samples into fp16 hi/lo arrays
    float wm = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    int xe = 0;
    if (wm > 0.f) {
        int E;
        frexpf(wm, &E);  // wm = f 2^E, f in [0.5, 1)
        xe = 11 - E;     // scaled maximum in [2^10, 2^11)
    }
#pragma unroll
    for (int q = 0; q < G::spt; ++q) {
        const int e = tid + 256 * q;
        if (e < G::span) {
            const float re = ldexpf(xv[q].x, xe), im = ldexpf(xv[q].y, xe);
            const _Float16 rh = (_Float16)re, ih = (_Float16)im;
            a_rh[e] = rh;
            a_rl[e] = (_Float16)(re - (float)rh);
            a_ih[e] = ih;
            a_il[e] = (_Float16)(im - (float)ih);
        }
    }
    // 4) B fragments in lane order: block (s, r, part) holds, for lane l, the 8 values
    //    B_r[32 s + 8 (l / 16) + j][l % 16], j < 8, i.e. a_r[kappa - u] (tap index kappa - u)
    for (int id = tid; id < G::ksteps * kMfOrders * 64; id += 256) {
        const int l = id & 63;
        const int r = (id >> 6) % kMfOrders;
        const int s = (id >> 6) / kMfOrders;
        const int u = l & 15;
        half8 hi, lo8;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int kk = 32 * s + 8 * (l >> 4) + j - u;  // tap index 0 .. 2H
            const float c = (kk >= 0 && kk < G::ntap) ? coef[r * G::ntap + kk] : 0.f;
            const _Float16 ch = (_Float16)c;
            hi[j] = ch;
            lo8[j] = (_Float16)(c - (float)ch);
        }
        half8 *blk = reinterpret_cast<half8 *>(bsm + ((s * kMfOrders + r) * 2) * 1024);
        blk[l] = hi;
        blk[64 + l] = lo8;
    }
    __syncthreads();

    const int64_t m0 = M0 + 256 * wave;
    if (m0 >= jb.n_out)
        return;  // no barrier follows

    // 5) the GEMM: 8 accumulators (4 orders x re/im), 24 MFMAs per 32-tap step
    floatx4 acc[kMfOrders][2];
#pragma unroll
    for (int r = 0; r < kMfOrders; ++r)
        acc[r][0] = acc[r][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int arow = 256 * wave + 16 * (lane & 15) + 8 * (lane >> 4);
#pragma unroll
    for (int s = 0; s < G::ksteps; ++s) {
        const int e = arow + 32 * s;
        const half8 xrh = *reinterpret_cast<const half8 *>(a_rh + e);
        const half8 xrl = *reinterpret_cast<const half8 *>(a_rl + e);
        const half8 xih = *reinterpret_cast<const half8 *>(a_ih + e);
        const half8 xil = *reinterpret_cast<const half8 *>(a_il + e);
        half8 bh[kMfOrders], bl[kMfOrders];
#pragma unroll
        for (int r = 0; r < kMfOrders; ++r) {
            const half8 *blk = reinterpret_cast<const half8 *>(bsm + ((s * kMfOrders + r) * 2) * 1024);
            bh[r] = blk[lane];
            bl[r] = blk[64 + lane];
        }
#pragma unroll
        for (int r = 0; r < kMfOrders; ++r) {
            acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xrh, bh[r], acc[r][0], 0, 0, 0);
            acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xih, bh[r], acc[r][1], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < kMfOrders; ++r) {
            acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xrh, bl[r], acc[r][0], 0, 0, 0);
            acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xih, bl[r], acc[r][1], 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < kMfOrders; ++r) {
            acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xrl, bh[r], acc[r][0], 0, 0, 0);
            acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xil, bh[r], acc[r][1], 0, 0, 0);
        }
    }

    // 6) lane holds Z_r[row 4 (l/16) + j][col l % 16]: output m = m0 + 16 row + col
    const float unscale = ldexpf(1.0f, -(xe + kCoefExp));
    const double inv_d = 1.0 / D;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t m = m0 + 16 * (4 * (lane >> 4) + j) + (lane & 15);
        if (m >= jb.n_out)
            continue;
        const double md = (double)m;
        const double sig = (__dmul_rn(alpha, md) - md) - Sd;  // exact, as in the direct form
        float2 out;
        if (sig == 0.0) {
            const int64_t src = m + S;
            out = (src >= 0 && src < jb.n_in) ? jb.x[src] : make_float2(0.f, 0.f);
        } else {
            const float z = (float)((sig - sc) * inv_d);
            float yr = acc[3][0][j], yi = acc[3][1][j];
#pragma unroll
            for (int r = 2; r >= 0; --r) {
                yr = fmaf(yr, z, acc[r][0][j]);
                yi = fmaf(yi, z, acc[r][1][j]);
            }
            out = make_float2(yr * unscale, yi * unscale);
        }
        jb.y[m] = out;
    }
}

// Chebyshev nodes of [-1, 1] and the inverse of their 4x4 Vandermonde matrix.
MfmaSincConst make_mfma_const()
{
    MfmaSincConst c{};
    double V[4][4], inv[4][8];
    for (int i = 0; i < 4; ++i) {
        c.node[i] = std::cos((2.0 * i + 1.0) * kPi / 8.0);
        for (int r = 0; r < 4; ++r)
            V[i][r] = std::pow(c.node[i], r);
    }
    // Gauss-Jordan on [V | I]; V[i][r] = z_i^r, so a = V^-1 h gives p(z) = sum_r a_r z^r
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j)
            inv[i][j] = j < 4 ? V[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int p = 0; p < 4; ++p) {
        int piv = p;
        for (int i = p + 1; i < 4; ++i)
            if (std::fabs(inv[i][p]) > std::fabs(inv[piv][p]))
                piv = i;
        for (int j = 0; j < 8; ++j)
            std::swap(inv[p][j], inv[piv][j]);
        const double d = inv[p][p];
        for (int j = 0; j < 8; ++j)
            inv[p][j] /= d;
        for (int i = 0; i < 4; ++i)
            if (i != p) {
                const double f = inv[i][p];
                for (int j = 0; j < 8; ++j)
                    inv[i][j] -= f * inv[p][j];
            }
    }
    for (int r = 0; r < 4; ++r)
        for (int i = 0; i < 4; ++i)
            c.vinv[r * 4 + i] = inv[r][4 + i];
    return c;
}

template <int H>
hipError_t launch_h(const SincJob *jobs_dev, const SincJob &inl, int njobs, int64_t nblk,
                    const KaiserPoly &kp, hipStream_t s)
{
    static const MfmaSincConst mc = make_mfma_const();
    static bool attr_set = false;
    const size_t lds = MfGeom<H>::bytes;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sinc_mfma<H>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_sinc_mfma<H>, dim3((unsigned)nblk, (unsigned)njobs), dim3(256), lds, s, jobs_dev,
                       inl, kp, mc);
    return hipGetLastError();
}

}  // namespace

bool sinc_mfma_eligible(double alpha, const rc_sinc &k)
{
    return k.window == RC_WIN_KAISER && (k.half_width == 64 || k.half_width == 128) &&
           std::fabs(alpha - 1.0) <= kSincMfmaMaxEps;
}

hipError_t launch_sinc_mfma(const SincJob *jobs_dev, const SincJob *job_inline, int njobs, int64_t max_out,
                            int half_width, const KaiserPoly &kp, hipStream_t s, Profiler *prof)
{
    if (njobs <= 0 || max_out <= 0)
        return hipSuccess;
    const int64_t nblk = (max_out + kMfOut - 1) / kMfOut;
    if (nblk > 0x7fffffff || njobs > 65535)
        return hipErrorInvalidValue;
    const SincJob inl = job_inline ? *job_inline : SincJob{};
    if (prof)
        prof->begin(kKSincMfma, s);
    hipError_t e = half_width == 64 ? launch_h<64>(jobs_dev, inl, njobs, nblk, kp, s)
                                    : launch_h<128>(jobs_dev, inl, njobs, nblk, kp, s);
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace rc
