// fft.hip -- ionospheric operator of Eq (15)/(16) for gfx950:
//   y = IDFT( DFT(x) * exp(s i 4 pi K2 / (c f_k)) ),  f_k = carrier + fs * fftfreq(n)[k].
//
// An n-point transform is split into levels L_0 x ... x L_{d-1} (row-major, last level
// contiguous, <= 4096 points; strided levels <= 256 points):
//   forward strided passes (i = 0 .. d-2): length-L_i DFT along level i, then the twiddle
//     exp(-2 pi i k_i n' / nsub_i) with n' the flat position inside the lower levels;
//   one contiguous pass: forward DFT of each row, the dispersive phase of its bins (float64
//     argument in quarter turns, float32 polynomial for the remainder), inverse DFT;
//   inverse strided passes (i = d-2 .. 0): conjugate twiddle, inverse DFT, 1/n in the last.
// The frequency of a bin never leaves the digit-reversed order of the levels, so no
// reordering pass exists.  Every pass works on a 4096-sample tile with coalesced accesses
// (levels of 16 points or fewer in registers, one column per thread; others through LDS),
// runs Stockham radix-16/8/4/2 stages and writes the tile back to the same place: every pass
// after the first runs in place on y.  Twiddles are products of a few base roots, taken from a
// float64-built table or from sincospi of exact float32 arguments.
#include <cmath>
#include <vector>

#include "rc_internal.h"

namespace rc {

namespace {

// A value every lane of the wave holds alike (a job descriptor of a block), moved into scalar
// registers so that it costs no vector registers while it stays live.
template <class T> __device__ __forceinline__ T wave_uniform(const T &x)
{
    static_assert(sizeof(T) % 4 == 0, "whole dwords only");
    T y;
    const int *src = reinterpret_cast<const int *>(&x);
    int *dst = reinterpret_cast<int *>(&y);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i)
        dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return y;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// z * (S i), S = -1 or +1
template <int S> __device__ __forceinline__ float2 mul_si(float2 z)
{
    return S < 0 ? make_float2(z.y, -z.x) : make_float2(-z.y, z.x);
}

template <int S> __device__ __forceinline__ void dft2(float2 *v)
{
    const float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <int S> __device__ __forceinline__ void dft4v(float2 &v0, float2 &v1, float2 &v2, float2 &v3)
{
    const float2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_si<S>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <int S> __device__ __forceinline__ void dft4(float2 *v) { dft4v<S>(v[0], v[1], v[2], v[3]); }

template <int S> __device__ __forceinline__ void dft8(float2 *v)
{
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4v<S>(e0, e1, e2, e3);
    dft4v<S>(o0, o1, o2, o3);
    const float r = 0.70710678118654752f;
    o1 = cmul(o1, make_float2(r, S * r));   // W8^1
    o2 = mul_si<S>(o2);                      // W8^2
    o3 = cmul(o3, make_float2(-r, S * r));  // W8^3
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <int S> __device__ __forceinline__ void dft16(float2 *v)
{
    // n = 4 n1 + n2, k = k1 + 4 k2:  X[k] = sum_n2 W16^(n2 k1) W4^(n2 k2) sum_n1 x[n] W4^(n1 k1)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
        dft4v<S>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);  // v[n2 + 4 k1]
    const float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, c2 = 0.70710678118654752f;
    v[5] = cmul(v[5], make_float2(c1, S * s1));     // W^1
    v[9] = cmul(v[9], make_float2(c2, S * c2));     // W^2
    v[13] = cmul(v[13], make_float2(s1, S * c1));   // W^3
    v[6] = cmul(v[6], make_float2(c2, S * c2));     // W^2
    v[10] = mul_si<S>(v[10]);                       // W^4
    v[14] = cmul(v[14], make_float2(-c2, S * c2));  // W^6
    v[7] = cmul(v[7], make_float2(s1, S * c1));     // W^3
    v[11] = cmul(v[11], make_float2(-c2, S * c2));  // W^6
    v[15] = cmul(v[15], make_float2(-c1, -S * s1)); // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
        dft4v<S>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);  // v[4 k1 + k2] = X[k1 + 4 k2]
    float2 t;
#define RC_SWAP(a, b) (t = v[a], v[a] = v[b], v[b] = t)
    RC_SWAP(1, 4); RC_SWAP(2, 8); RC_SWAP(3, 12); RC_SWAP(6, 9); RC_SWAP(7, 13); RC_SWAP(11, 14);
#undef RC_SWAP
}

template <int R, int S> __device__ __forceinline__ void dftR(float2 *v)
{
    if constexpr (R == 2) dft2<S>(v);
    else if constexpr (R == 4) dft4<S>(v);
    else if constexpr (R == 8) dft8<S>(v);
    else dft16<S>(v);
}

// exp(S 2 pi i q / M), M = 2^log2M <= 2^24: sincospi of an exact float32 argument.
template <int S>
__device__ __forceinline__ float2 unit_root(int64_t q, int log2M)
{
    const float th = (float)(q & ((int64_t(1) << log2M) - 1)) * ldexpf(2.0f, -log2M);
    float sn, cs;
    sincospif(th, &sn, &cs);
    return make_float2(cs, S * sn);
}

// Bases exp(S 2 pi i 2^t m / M), t = 0..3 (those below R), of the stage twiddle
// exp(S 2 pi i q m / M), M a power of two <= 2^24: sincospi of exact float32 arguments.
template <int R, int S>
__device__ __forceinline__ void twiddle_bases(float2 *b, int64_t m, int log2M)
{
    const int64_t mask = (int64_t(1) << log2M) - 1;
    const float scale = ldexpf(2.0f, -log2M);  // 2 / M, exact
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if ((1 << t) < R) {
            const float th = (float)((m << t) & mask) * scale;  // exact: < 2^24 times a power of two
            float sn, cs;
            sincospif(th, &sn, &cs);
            b[t] = make_float2(cs, S * sn);
        }
    }
}

// v[q] *= b^q for q = 1 .. R-1, where b[t] holds the 2^t-th power: every other power is a product
// of at most four bases (error within ~5 ulp).  No table gathers: a table indexed by q m scatters
// a wave's loads over as many cache lines as it has lanes.
template <int R>
__device__ __forceinline__ void twiddle_apply(float2 *v, const float2 *b)
{
    float2 w3 = make_float2(1.f, 0.f), w5 = w3, w6 = w3, w7 = w3;
    if (R > 1) v[1] = cmul(v[1], b[0]);
    if (R > 2) {
        v[2] = cmul(v[2], b[1]);
        w3 = cmul(b[0], b[1]);
        v[3] = cmul(v[3], w3);
    }
    if (R > 4) {
        v[4] = cmul(v[4], b[2]);
        w5 = cmul(b[0], b[2]);
        w6 = cmul(b[1], b[2]);
        w7 = cmul(w3, b[2]);
        v[5] = cmul(v[5], w5);
        v[6] = cmul(v[6], w6);
        v[7] = cmul(v[7], w7);
    }
    if (R > 8) {
        v[8] = cmul(v[8], b[3]);
        v[9] = cmul(v[9], cmul(b[0], b[3]));
        v[10] = cmul(v[10], cmul(b[1], b[3]));
        v[11] = cmul(v[11], cmul(w3, b[3]));
        v[12] = cmul(v[12], cmul(b[2], b[3]));
        v[13] = cmul(v[13], cmul(w5, b[3]));
        v[14] = cmul(v[14], cmul(w6, b[3]));
        v[15] = cmul(v[15], cmul(w7, b[3]));
    }
}

// v[q] *= exp(S 2 pi i q m / M) for q = 1 .. R-1.
template <int R, int S>
__device__ __forceinline__ void twiddle_powers(float2 *v, int64_t m, int log2M)
{
    float2 b[4];
    twiddle_bases<R, S>(b, m, log2M);
    twiddle_apply<R>(v, b);
}

// LDS layout of a 4096-sample tile holding C lines of length L: element (c, l) at
// c*L + l (rows, "lc") or l*C + c (columns), with one pad slot per 16 samples.
__device__ __forceinline__ int tidx(int c, int l, int log2L, int log2C, bool lc)
{
    const int a = lc ? ((c << log2L) + l) : ((l << log2C) + c);
    return a + (a >> 4);
}
constexpr int kLdsSlots = kFftTile + kFftTile / 16;

// One Stockham radix-R stage over every line of the tile (Ns = product of earlier radices).
template <int R, int S>
__device__ __forceinline__ void stage(float2 *lds, int log2L, int log2C, bool lc, int Ns,
                                      const float2 *__restrict__ tw, int tid)
{
    constexpr int PER = 16 / R;
    const int log2BL = log2L - (R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4);
    const int BL = 1 << log2BL;  // butterflies per line
    float2 v[PER][R];
    int cc[PER], jj[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * kFftThreads;
        int c, j;
        if (lc) {
            c = b >> log2BL;
            j = b & (BL - 1);
        } else {
            c = b & ((1 << log2C) - 1);
            j = b >> log2C;
        }
        cc[p] = c;
        jj[p] = j;
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[p][r] = lds[tidx(c, j + r * BL, log2L, log2C, lc)];
        if (Ns > 1) {
            // twiddle W^(r k step), r < R: the log2 R bases W^(2^t k step) from the table (a
            // gather each), the other powers as products of them
            const int k = j & (Ns - 1);
            const int step = kFftTile / (Ns * R);
            constexpr int NB = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
            float2 bb[4];
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                float2 w = gmem(tw)[((k * step) << t) & (kFftTile - 1)];
                if (S > 0)
                    w.y = -w.y;
                bb[t] = w;
            }
            twiddle_apply<R>(v[p], bb);
        }
        dftR<R, S>(v[p]);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int k = jj[p] & (Ns - 1);
        const int base = (jj[p] - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r)
            lds[tidx(cc[p], base + r * Ns, log2L, log2C, lc)] = v[p][r];
    }
    __syncthreads();
}

// Full length-L DFT (sign S) of every line of the tile; natural order in and out.
template <int S>
__device__ void fft_tile(float2 *lds, int log2L, int log2C, bool lc, const float2 *__restrict__ tw,
                         int tid)
{
    int Ns = 1;
    const int rem = log2L & 3;
    if (rem == 1) {
        stage<2, S>(lds, log2L, log2C, lc, Ns, tw, tid);
        Ns = 2;
    } else if (rem == 2) {
        stage<4, S>(lds, log2L, log2C, lc, Ns, tw, tid);
        Ns = 4;
    } else if (rem == 3) {
        stage<8, S>(lds, log2L, log2C, lc, Ns, tw, tid);
        Ns = 8;
    }
    for (int s = 0; s < (log2L >> 2); ++s) {
        stage<16, S>(lds, log2L, log2C, lc, Ns, tw, tid);
        Ns <<= 4;
    }
}

struct StridedArgs {
    const IonoJob *jobs;
    IonoJob inl;
    int njobs;
    int log2L, log2C;
    int64_t inner;          // samples below this level (line stride)
    int log2cb;             // log2(inner / columns per block)
    int log2pp;             // log2(outer * inner / columns per block): blocks per pulse
    const float2 *tw4096;
    int log2nsub;           // log2(L * inner)
    bool from_x;            // first pass reads job.x
    bool reverse;           // walk the blocks from the last (see pass_order)
    float scale;            // applied after an inverse pass (1/n in the last one)
};

// Consecutive passes walk the batch in opposite directions: a pass then starts on the samples
// the previous one wrote last, which are still in the memory-side cache.  The block order is
// the only difference; every block does the same work either way.
__device__ __forceinline__ int64_t pass_order(bool reverse)
{
    return reverse ? (int64_t)gridDim.x - 1 - (int64_t)blockIdx.x : (int64_t)blockIdx.x;
}

// Strided level of length L <= 16 (one radix stage): each thread owns one column and keeps
// its L samples in registers -- no LDS, no barrier.  A block covers 256 adjacent columns.
template <int R, int S>
__global__ void __launch_bounds__(kFftThreads) k_fft_strided_reg(StridedArgs a)
{
    const int64_t blk = pass_order(a.reverse);
    const int p = (int)(blk >> a.log2pp);
    const int64_t rem = blk & ((int64_t(1) << a.log2pp) - 1);
    const int64_t o = rem >> a.log2cb;
    const int64_t col = ((rem & ((int64_t(1) << a.log2cb) - 1)) << 8) + threadIdx.x;  // n'
    const IonoJob jb = a.jobs ? gload(a.jobs, p) : a.inl;
    const int64_t base = o * (R * a.inner) + col;
    const auto src = gmem(a.from_x ? jb.x : jb.y);
    float2 v[R];
#pragma unroll
    for (int l = 0; l < R; ++l)
        v[l] = src[base + l * a.inner];
    if (S > 0)
        twiddle_powers<R, +1>(v, col, a.log2nsub);
    dftR<R, S>(v);
    if (S < 0) {
        twiddle_powers<R, -1>(v, col, a.log2nsub);
    } else if (a.scale != 1.0f) {
#pragma unroll
        for (int l = 0; l < R; ++l) {
            v[l].x *= a.scale;
            v[l].y *= a.scale;
        }
    }
#pragma unroll
    for (int l = 0; l < R; ++l)
        store_nt(jb.y + base + l * a.inner, v[l]);
}

// Strided level of length 32..256: lines of length L along stride `inner`; the LDS tile holds
// C = 4096/L adjacent columns.  Thread t owns the 16 tile elements of column c = t % C at rows
// l0 + D k (l0 = t / C, D = 256 / C, k < 16); their twiddles exp(S 2 pi i l n' / nsub), n' the
// column's position, are b0 (b^k), b0 = w^(l0 n'), b = w^(D n'): two sincospi-based bases and
// products instead of one sincospi per element.
template <int S>
__device__ __forceinline__ void strided_twiddles(float2 *v, int l0, int D, int64_t np, int log2nsub)
{
    const float2 b0 = unit_root<S>((int64_t)l0 * np, log2nsub);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        v[k] = cmul(v[k], b0);
    float2 bb[4];
    twiddle_bases<16, S>(bb, (int64_t)D * np, log2nsub);
    twiddle_apply<16>(v, bb);
}

template <int S>
__global__ void __launch_bounds__(kFftThreads) k_fft_strided(StridedArgs a)
{
    __shared__ float2 lds[kLdsSlots];
    const int tid = threadIdx.x;
    const int64_t blk = pass_order(a.reverse);
    const int p = (int)(blk >> a.log2pp);
    const int64_t rem = blk & ((int64_t(1) << a.log2pp) - 1);
    const int64_t o = rem >> a.log2cb;
    const int64_t cb = rem & ((int64_t(1) << a.log2cb) - 1);
    const IonoJob jb = a.jobs ? gload(a.jobs, p) : a.inl;
    const int L = 1 << a.log2L, C = 1 << a.log2C;
    const int64_t base = o * ((int64_t)L * a.inner) + cb * C;
    const int c = tid & (C - 1), l0 = tid >> a.log2C, D = kFftThreads >> a.log2C;
    const int64_t np = cb * C + c;  // n': the column's position inside the lower levels
    const auto src = gmem(a.from_x ? jb.x : jb.y) + base + c;
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        v[k] = src[(int64_t)(l0 + D * k) * a.inner];
    if (S > 0)  // inverse: conjugate twiddle before the DFT along the level
        strided_twiddles<+1>(v, l0, D, np, a.log2nsub);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        lds[tidx(c, l0 + D * k, a.log2L, a.log2C, false)] = v[k];
    __syncthreads();
    fft_tile<S>(lds, a.log2L, a.log2C, false, a.tw4096, tid);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        v[k] = lds[tidx(c, l0 + D * k, a.log2L, a.log2C, false)];
    if (S < 0) {  // forward: twiddle after the DFT, k = l, n' = column position
        strided_twiddles<-1>(v, l0, D, np, a.log2nsub);
    } else if (a.scale != 1.0f) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k].x *= a.scale;
            v[k].y *= a.scale;
        }
    }
    const auto dst = gmem(jb.y) + base + c;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        dst[(int64_t)(l0 + D * k) * a.inner] = v[k];
}

struct RowArgs {
    const IonoJob *jobs;
    IonoJob inl;
    int njobs;
    int log2L, log2C;
    int log2rpp;              // log2(rows per pulse) = log2(n / L)
    int64_t n;
    int levels;
    int len[kFftMaxLevels];   // level lengths (the last is L)
    const float2 *tw4096;
    bool from_x;
    bool fwd_only;            // store the spectrum (native order) after the forward transform
    bool reverse;             // walk the rows from the last (see pass_order)
    float scale;              // 1/n when this is the only pass, else 1
};

// (cos pi w / 2, sin pi w / 2) for |w| <= 1/2 quarter turn: with u = w^2, w S(u) and 1 + u C(u),
// S and C cubics fitted (weighted Remez exchange on u in [0, 1/4], the coefficients rounded to
// float32 one at a time with the rest refitted; fit_cis_quarter.py) to an absolute error below
// 5.1e-9 (sin) and 4.1e-10 (cos); float32 evaluation stays within 7e-8 and 2 ulp of the true values.
__device__ __forceinline__ float2 cis_quarter(float w)
{
    const float u = w * w;
    float ps = fmaf(u, -0x1.2a7638p-8f, 0x1.46496cp-4f);
    ps = fmaf(u, ps, -0x1.4abb68p-1f);
    ps = fmaf(u, ps, 0x1.921fb4p+0f);
    float pc = fmaf(u, 0x1.d47d46p-11f, -0x1.55b146p-6f);
    pc = fmaf(u, pc, 0x1.03c1aep-2f);
    pc = fmaf(u, pc, -0x1.3bd3ccp+0f);
    return make_float2(fmaf(u, pc, 1.0f), w * ps);
}

// Per-job constants of the dispersive phase of Eq (15)/(16): in quarter turns the phase at bin
// frequency f is c4 / f, with f = carrier + fs_n kk for the signed bin index kk (fs_n = fs / n).
// With xprec the quotient is (c4 n) / (carrier n + fs kk) in double-double arithmetic: c4n and
// cn are the exact products c4 n and carrier n as unevaluated sums hi + lo.
struct PhaseK {
    double c4, carrier, fs_n;
    double c4n_hi, c4n_lo, cn_hi, cn_lo, fs;
    bool xprec;
};

__device__ __forceinline__ PhaseK phase_consts(const IonoJob &jb, int64_t n)
{
    PhaseK P;
    const double nd = (double)n;
    P.c4 = jb.phase.hi;
    P.carrier = jb.carrier;
    P.fs_n = jb.fs * (1.0 / nd);
    P.fs = jb.fs;
    P.xprec = jb.phase.xprec != 0;
    P.c4n_hi = jb.phase.hi * nd;
    P.c4n_lo = fma(jb.phase.hi, nd, -P.c4n_hi) + jb.phase.lo * nd;
    P.cn_hi = jb.carrier * nd;
    P.cn_lo = fma(jb.carrier, nd, -P.cn_hi);
    return P;
}

__device__ __forceinline__ float2 phase_at(const PhaseK &P, int64_t kk)
{
    double f, rf, t4, t4_lo = 0.0;
    if (!P.xprec) {
        f = fma(P.fs_n, (double)kk, P.carrier);
        // t4 = c4 / f quarter turns.  1/f comes from the hardware reciprocal (relative error
        // below 2^-24 on gfx950) and one Newton step (below 2^-48); the quotient then takes one
        // residual correction, t4 += (c4 - t4 f) / f, which leaves it within a few ulp of c4 / f.
        // Without xprec |t4| < 2^26, so that is within 2^-24 quarter turn.
        rf = __builtin_amdgcn_rcp(f);
        rf = fma(rf, fma(-f, rf, 1.0), rf);
        t4 = P.c4 * rf;
        t4 = fma(fma(-t4, f, P.c4), rf, t4);
    } else {
        // d = carrier n + fs kk as hi + lo: fs kk exactly (two products), then a two-sum with
        // carrier n.  d is n f, so t4 = (c4 n) / d.
        const double k = (double)kk;
        const double p = P.fs * k;
        const double pe = fma(P.fs, k, -p);
        const double sm = P.cn_hi + p;
        const double bb = sm - P.cn_hi;
        const double l = ((P.cn_hi - (sm - bb)) + (p - bb)) + (pe + P.cn_lo);
        f = sm + l;
        const double f_lo = l - (f - sm);
        rf = __builtin_amdgcn_rcp(f);
        rf = fma(rf, fma(-f, rf, 1.0), rf);
        t4 = P.c4n_hi * rf;
        t4 = fma(fma(-t4, f, P.c4n_hi), rf, t4);
        // The remainder c4n - t4 d, with the product t4 f_hi exact through the fma; the quotient
        // is t4 + remainder / d to about 2^-100 relative.
        double r = fma(-t4, f, P.c4n_hi) + P.c4n_lo;
        r = fma(-t4, f_lo, r);
        t4_lo = r * rf;
    }
    // t4 splits exactly into a whole number n4 and a remainder w in [-1/2, 1/2] (n4 and t4 - n4
    // are exact for |t4| < 2^52); cis(pi w / 2) in float32 is then turned by n4 quarter turns.
    const double n4 = rint(t4);
    const float2 w = cis_quarter((float)((t4 - n4) + t4_lo));
    // n4 mod 4, exact in float64: n4/4, its floor and 4 floor(n4/4) are all exact integers.
    const int quad = (int)(n4 - 4.0 * floor(0.25 * n4));
    const float c = (quad & 1) ? -w.y : w.x;  // (c, s) turned by quad * 90 degrees
    const float sn = (quad & 1) ? w.x : w.y;
    if (f == 0.0)
        return make_float2(1.f, 0.f);
    return (quad & 2) ? make_float2(-c, -sn) : make_float2(c, sn);
}

// phase_at without xprec, in fewer instructions and with the same result: |n4| < 2^26 there,
// so n4 converts to int exactly and its two low bits are n4 mod 4; the quarter turns are applied
// by swapping (bit 0) and by flipping both signs (bit 1); f == 0 is selected, not branched to.
__device__ __forceinline__ float2 phase_fast(const PhaseK &P, int kk)
{
    const double f = fma(P.fs_n, (double)kk, P.carrier);
    double rf = __builtin_amdgcn_rcp(f);
    rf = fma(rf, fma(-f, rf, 1.0), rf);
    double t4 = P.c4 * rf;
    t4 = fma(fma(-t4, f, P.c4), rf, t4);
    const double n4 = rint(t4);
    const float2 w = cis_quarter((float)(t4 - n4));
    const int quad = (int)n4;
    const bool odd = quad & 1;
    const unsigned flip = ((unsigned)quad & 2u) << 30;  // sign bit when quad & 2
    float c = odd ? -w.y : w.x;
    float sn = odd ? w.x : w.y;
    c = __uint_as_float(__float_as_uint(c) ^ flip);
    sn = __uint_as_float(__float_as_uint(sn) ^ flip);
    return f == 0.0 ? make_float2(1.f, 0.f) : make_float2(c, sn);
}

__device__ __forceinline__ float2 iono_phase(const IonoJob &jb, int64_t k, int64_t n)
{
    const int64_t kk = (k < (n + 1) / 2) ? k : k - n;
    return phase_at(phase_consts(jb, n), kk);
}

// The factor of bin k (table entry t of the job's native order): the table value (conjugated
// if asked) times the dispersive phase, either of them 1 when absent.
__device__ __forceinline__ float2 bin_factor(const IonoJob &jb, int64_t t, int64_t k, int64_t n)
{
    float2 f = make_float2(1.f, 0.f);
    if (jb.mult) {
        f = gload(jb.mult, t);
        if (jb.conj_mult)
            f.y = -f.y;
    }
    if (jb.phase.hi != 0.0) {
        const float2 w = iono_phase(jb, k, n);
        f = jb.mult ? cmul(f, w) : w;
    }
    return f;
}

// One radix-16 Stockham stage of a 4096-point row held as 16 samples per thread
// (thread j owns positions j + 256 q).  Ns = 16^stage; the output leaves through LDS,
// except for the last stage, whose outputs j + 256 q are already in place.
__device__ __forceinline__ int rpad(int a) { return a + (a >> 4); }

// Full 4096-point DFT of the thread-distributed row: in v[q] = x[j + 256 q], out v[q] = X[j + 256 q].
// b2 and b3 are the forward twiddle bases of stages 2 and 3 (m = 16 (j % 16) and m = j over 4096);
// the inverse uses their conjugates, so one set of sincospi serves both transforms of a row.
template <int S>
__device__ __forceinline__ void row4096(float2 *v, float2 *lds, int j, const float2 *b2, const float2 *b3)
{
    float2 w[4];
    // stage 1 (Ns = 1): outputs at 16 j + q
    dftR<16, S>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q)
        lds[rpad(16 * j + q)] = v[q];
    __syncthreads();
    // stage 2 (Ns = 16): inputs j + 256 q, outputs (j / 16) * 256 + j % 16 + 16 q
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = lds[rpad(j + 256 * q)];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        w[t] = make_float2(b2[t].x, S < 0 ? b2[t].y : -b2[t].y);
    twiddle_apply<16>(v, w);
    dftR<16, S>(v);
    __syncthreads();
    const int base = ((j >> 4) << 8) + (j & 15);
#pragma unroll
    for (int q = 0; q < 16; ++q)
        lds[rpad(base + 16 * q)] = v[q];
    __syncthreads();
    // stage 3 (Ns = 256): inputs j + 256 q, outputs j + 256 q
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = lds[rpad(j + 256 * q)];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        w[t] = make_float2(b3[t].x, S < 0 ? b3[t].y : -b3[t].y);
    twiddle_apply<16>(v, w);
    dftR<16, S>(v);
    __syncthreads();  // LDS free for the next transform
}

// Row position l of row r of a 4096-point contiguous level holds bin kout + mult l, where kout is
// the digit-reversed row index and mult = n / 4096.
__device__ __forceinline__ void row_bin_origin(const RowArgs &a, int64_t r, int &kout, int &mult)
{
    int64_t ko = 0, m = 1, rr = r;
    int64_t digits[kFftMaxLevels];
    for (int i = a.levels - 2; i >= 0; --i) {
        digits[i] = rr & (a.len[i] - 1);
        rr >>= __ffs(a.len[i]) - 1;
    }
    for (int i = 0; i < a.levels - 1; ++i) {
        ko += digits[i] * m;
        m *= a.len[i];
    }
    kout = (int)ko;  // n <= 2^24
    mult = (int)m;
}

// Dispersive phase of the bin at row position l (see row_bin_origin), with the signed frequency
// index of the bins above n / 2.
__device__ __forceinline__ float2 row_phase(const PhaseK &pk, int kout, int mult, int l, int n)
{
    const int k = kout + mult * l;
    return phase_at(pk, k < (n + 1) / 2 ? k : k - n);
}

__device__ __forceinline__ float2 row_phase_fast(const PhaseK &pk, int kout, int mult, int l, int n)
{
    const int k = kout + mult * l;
    return phase_fast(pk, k < (n + 1) / 2 ? k : k - n);
}

// Contiguous level of 4096 points, one row per block: forward DFT, the per-bin factor, inverse
// DFT.  F selects the factor (see RowFactor).  The correlation variant holds the table across the
// forward transform and evaluates the phases after it: it needs more than 128 registers, so it
// runs at three blocks per CU instead of four.  Scaled: the outputs take a.scale (not 1).
template <int F, bool Scaled>
__global__ void __launch_bounds__(kFftThreads, F == kRowTablePhase ? 3 : 4) k_fft_row4096_iono(RowArgs a)
{
    __shared__ float2 lds[kLdsSlots];
    const int j = threadIdx.x;
    const int64_t g = pass_order(a.reverse);
    const int p = (int)(g >> a.log2rpp);
    const int64_t r = g & ((int64_t(1) << a.log2rpp) - 1);
    const IonoJob jb = wave_uniform(a.jobs ? gload(a.jobs, p) : a.inl);
    const auto src = gmem(a.from_x ? jb.x : jb.y) + (r << 12);
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = src[j + 256 * q];
    // forward twiddle bases W^(2^t m), W = exp(-2 pi i / 4096), from the float64-built table
    // (read while the row's loads are in flight): m = 16 (j % 16) for stage 2, m = j for stage 3
    float2 b2[4], b3[4];
    const auto tw = gmem(a.tw4096);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        b2[t] = tw[((16 * (j & 15)) << t) & (kFftTile - 1)];
        b3[t] = tw[(j << t) & (kFftTile - 1)];
    }
    // The per-bin factors depend on bin indices only: the phases are computed (or the table read)
    // while the row's samples are still in flight.  With both (F == kRowTablePhase) the table is
    // read here and the phase evaluated after the forward transform.
    float2 ph[16];
    if (!a.fwd_only) {
        if (F == kRowTablePhase || jb.mult) {  // the table is in this row's native order
            const auto tab = gmem(jb.mult) + (r << 12);
#pragma unroll
            for (int q = 0; q < 16; ++q)
                ph[q] = tab[j + 256 * q];
        } else {
            int kout, mult;
            row_bin_origin(a, r, kout, mult);
            const PhaseK pk = phase_consts(jb, a.n);
            if (pk.xprec) {  // uniform over the workgroup
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    ph[q] = row_phase(pk, kout, mult, j + 256 * q, (int)a.n);
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    ph[q] = row_phase_fast(pk, kout, mult, j + 256 * q, (int)a.n);
            }
        }
    }
    row4096<-1>(v, lds, j, b2, b3);
    if (a.fwd_only) {
        const auto dst = gmem(jb.y) + (r << 12);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            dst[j + 256 * q] = Scaled ? make_float2(v[q].x * a.scale, v[q].y * a.scale) : v[q];
        return;  // uniform over the workgroup
    }
    if constexpr (F == kRowTablePhase) {
        // a correlation: the table (conjugated if asked) times the phase, four bins at a time,
        // fenced from the scheduler so that the float64 evaluations do not pile up and spill
        int kout, mult;
        row_bin_origin(a, r, kout, mult);
        const PhaseK pk = phase_consts(jb, a.n);
#pragma unroll
        for (int q0 = 0; q0 < 16; q0 += 4) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = q0; q < q0 + 4; ++q) {
                float2 t = ph[q];
                if (jb.conj_mult)
                    t.y = -t.y;
                v[q] = cmul(v[q], cmul(t, row_phase(pk, kout, mult, j + 256 * q, (int)a.n)));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = cmul(v[q], ph[q]);
    }
    row4096<+1>(v, lds, j, b2, b3);
#pragma unroll
    for (int q = 0; q < 16; ++q)
        store_nt(jb.y + (r << 12) + j + 256 * q, Scaled ? make_float2(v[q].x * a.scale, v[q].y * a.scale) : v[q]);
}

// Single-level transform of n = L < 4096 points: the tile holds C = 4096/L whole pulses.
__global__ void __launch_bounds__(kFftThreads) k_fft_rows_iono(RowArgs a)
{
    __shared__ float2 lds[kLdsSlots];
    const int tid = threadIdx.x;
    const int L = 1 << a.log2L, C = 1 << a.log2C;
    const int g0 = (int)pass_order(a.reverse) * C;  // first pulse of the tile
    for (int e = tid; e < kFftTile; e += kFftThreads) {
        const int c = e >> a.log2L, l = e & (L - 1);
        const int g = g0 + c;
        float2 v = make_float2(0.f, 0.f);
        if (g < a.njobs) {
            const IonoJob jb = a.jobs ? gload(a.jobs, g) : a.inl;
            v = gmem(a.from_x ? jb.x : jb.y)[l];
        }
        lds[tidx(c, l, a.log2L, a.log2C, true)] = v;
    }
    __syncthreads();
    fft_tile<-1>(lds, a.log2L, a.log2C, true, a.tw4096, tid);
    for (int e = tid; e < kFftTile; e += kFftThreads) {
        const int c = e >> a.log2L, l = e & (L - 1);
        const int g = g0 + c;
        if (g >= a.njobs)
            continue;
        const IonoJob jb = a.jobs ? gload(a.jobs, g) : a.inl;
        const int idx = tidx(c, l, a.log2L, a.log2C, true);
        if (a.fwd_only) {
            float2 v = lds[idx];
            v.x *= a.scale;
            v.y *= a.scale;
            gmem(jb.y)[l] = v;
        } else {
            lds[idx] = cmul(lds[idx], bin_factor(jb, l, l, a.n));
        }
    }
    if (a.fwd_only)
        return;  // uniform over the workgroup
    __syncthreads();
    fft_tile<+1>(lds, a.log2L, a.log2C, true, a.tw4096, tid);
    for (int e = tid; e < kFftTile; e += kFftThreads) {
        const int c = e >> a.log2L, l = e & (L - 1);
        const int g = g0 + c;
        if (g >= a.njobs)
            continue;
        const IonoJob jb = a.jobs ? gload(a.jobs, g) : a.inl;
        float2 v = lds[tidx(c, l, a.log2L, a.log2C, true)];
        v.x *= a.scale;
        v.y *= a.scale;
        gmem(jb.y)[l] = v;
    }
}

int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v)
        ++l;
    return l;
}

hipError_t upload_table(const std::vector<float2> &h, float2 **dev, std::vector<void *> &allocs)
{
    hipError_t e = hipMalloc(dev, h.size() * sizeof(float2));
    if (e != hipSuccess)
        return e;
    allocs.push_back(*dev);
    return hipMemcpy(*dev, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice);
}

// exp(-2 pi i q / m) for q = 0 .. count-1 with q*step exact, rounded once to float32.
std::vector<float2> twiddle_table(int64_t count, int64_t step, int64_t m)
{
    std::vector<float2> t((size_t)count);
    for (int64_t q = 0; q < count; ++q) {
        const int64_t r = (q * step) % m;
        const double a = -2.0 * kPi * (double)r / (double)m;
        t[(size_t)q] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    return t;
}

}  // namespace

hipError_t make_base_twiddles(float2 **dev)
{
    std::vector<void *> unused;
    return upload_table(twiddle_table(kFftTile, 1, kFftTile), dev, unused);
}

hipError_t build_fft_plan(int64_t n, FftPlan &plan, std::vector<void *> &allocs)
{
    plan = FftPlan{};
    plan.n = n;
    const int p = ilog2(n);
    if ((int64_t(1) << p) != n || p > 24)  // twiddle arguments stay exact up to 2^24
        return hipErrorInvalidValue;
    if (p <= 12) {
        plan.levels = 1;
        plan.len[0] = (int)n;
    } else {
        // strided levels of up to 256 points (fewer passes; a 2^24 transform measured faster as
        // 256 x 16 x 4096 than as 16 x 16 x 16 x 4096, whose first pass strides 8 MB)
        int rest = p - 12;
        int d = 0;
        while (rest > 0) {
            const int s = rest < 8 ? rest : 8;
            plan.len[d++] = 1 << s;
            rest -= s;
        }
        if (d + 1 > kFftMaxLevels)
            return hipErrorInvalidValue;
        plan.len[d++] = kFftTile;
        plan.levels = d;
    }
    for (int i = 0; i < plan.levels; ++i)
        plan.log2len[i] = ilog2(plan.len[i]);
    return hipSuccess;
}

hipError_t build_fft_plan_levels(int64_t n, const std::vector<int> &strided, FftPlan &plan)
{
    plan = FftPlan{};
    plan.n = n;
    if (ilog2(n) > 24 || (int64_t(1) << ilog2(n)) != n || n <= kFftTile || strided.empty() ||
        (int)strided.size() + 1 > kFftMaxLevels)
        return hipErrorInvalidValue;
    int64_t prod = kFftTile;
    for (int L : strided) {
        if (L < 2 || L > 256 || (L & (L - 1)) != 0)
            return hipErrorInvalidValue;
        prod *= L;
    }
    if (prod != n)
        return hipErrorInvalidValue;
    int d = 0;
    for (int L : strided)
        plan.len[d++] = L;
    plan.len[d++] = kFftTile;
    plan.levels = d;
    for (int i = 0; i < plan.levels; ++i)
        plan.log2len[i] = ilog2(plan.len[i]);
    return hipSuccess;
}

namespace {

hipError_t launch_fft_impl(const FftPlan &plan, const float2 *tw4096, const IonoJob *jobs_dev,
                           const IonoJob *job_inline, int njobs, bool fwd_only, int factor, hipStream_t s,
                           Profiler *prof)
{
    if (njobs <= 0)
        return hipSuccess;
    const IonoJob inl = job_inline ? *job_inline : IonoJob{};
    const int d = plan.levels;
    const float inv_n = (float)(1.0 / (double)plan.n);
    int64_t inner[kFftMaxLevels], outer[kFftMaxLevels];
    {
        int64_t below = plan.n, above = 1;
        for (int i = 0; i < d; ++i) {
            below /= plan.len[i];
            inner[i] = below;
            outer[i] = above;
            above *= plan.len[i];
        }
    }
    int pass = 0;  // consecutive passes alternate their block order
    auto strided = [&](int i, bool inverse) -> hipError_t {
        StridedArgs a{};
        a.reverse = (pass++ & 1) != 0;
        a.jobs = jobs_dev;
        a.inl = inl;
        a.njobs = njobs;
        a.log2L = plan.log2len[i];
        a.inner = inner[i];
        a.tw4096 = tw4096;
        a.log2nsub = plan.log2len[i] + ilog2(inner[i]);
        a.from_x = (!inverse && i == 0);
        a.scale = (inverse && i == 0) ? inv_n : 1.0f;
        const bool reg = plan.len[i] <= 16;
        // columns per block: 256 threads x 1 column (register kernel) or the LDS tile width
        a.log2C = reg ? 8 : ilog2(kFftTile) - plan.log2len[i];
        a.log2cb = ilog2(inner[i]) - a.log2C;
        a.log2pp = ilog2(outer[i]) + a.log2cb;
        const int64_t blocks = (int64_t)njobs << a.log2pp;
        if (blocks > 0x7fffffff)
            return hipErrorInvalidValue;
        if (prof)
            prof->begin(inverse ? kKFftStridedInv : kKFftStridedFwd, s);
        const dim3 grid((unsigned)blocks), blk(kFftThreads);
        if (reg) {
            switch (plan.len[i] * (inverse ? 1 : -1)) {
            case -2: hipLaunchKernelGGL((k_fft_strided_reg<2, -1>), grid, blk, 0, s, a); break;
            case -4: hipLaunchKernelGGL((k_fft_strided_reg<4, -1>), grid, blk, 0, s, a); break;
            case -8: hipLaunchKernelGGL((k_fft_strided_reg<8, -1>), grid, blk, 0, s, a); break;
            case -16: hipLaunchKernelGGL((k_fft_strided_reg<16, -1>), grid, blk, 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_fft_strided_reg<2, 1>), grid, blk, 0, s, a); break;
            case 4: hipLaunchKernelGGL((k_fft_strided_reg<4, 1>), grid, blk, 0, s, a); break;
            case 8: hipLaunchKernelGGL((k_fft_strided_reg<8, 1>), grid, blk, 0, s, a); break;
            default: hipLaunchKernelGGL((k_fft_strided_reg<16, 1>), grid, blk, 0, s, a); break;
            }
        } else if (inverse) {
            hipLaunchKernelGGL(k_fft_strided<+1>, grid, blk, 0, s, a);
        } else {
            hipLaunchKernelGGL(k_fft_strided<-1>, grid, blk, 0, s, a);
        }
        const hipError_t e = hipGetLastError();
        if (prof)
            prof->end(s);
        return e;
    };
    for (int i = 0; i + 1 < d; ++i) {
        hipError_t e = strided(i, false);
        if (e != hipSuccess)
            return e;
    }
    {
        RowArgs a{};
        a.jobs = jobs_dev;
        a.inl = inl;
        a.njobs = njobs;
        a.log2L = plan.log2len[d - 1];
        a.log2C = ilog2(kFftTile) - a.log2L;
        a.log2rpp = ilog2(plan.n) - a.log2L;
        a.n = plan.n;
        a.levels = d;
        for (int i = 0; i < kFftMaxLevels; ++i)
            a.len[i] = plan.len[i];
        a.tw4096 = tw4096;
        a.from_x = (d == 1);
        a.fwd_only = fwd_only;
        a.reverse = (pass++ & 1) != 0;
        a.scale = (d == 1 && !fwd_only) ? inv_n : 1.0f;
        if (prof)
            prof->begin(kKFftRowsIono, s);
        if (a.log2L == 12) {
            const int64_t blocks = (int64_t)njobs << a.log2rpp;
            if (blocks > 0x7fffffff)
                return hipErrorInvalidValue;
            const dim3 grid((unsigned)blocks);
            const bool scaled = a.scale != 1.0f;
            if (factor == kRowTablePhase && scaled)
                hipLaunchKernelGGL((k_fft_row4096_iono<kRowTablePhase, true>), grid, dim3(kFftThreads), 0, s, a);
            else if (factor == kRowTablePhase)
                hipLaunchKernelGGL((k_fft_row4096_iono<kRowTablePhase, false>), grid, dim3(kFftThreads), 0, s, a);
            else if (scaled)
                hipLaunchKernelGGL((k_fft_row4096_iono<kRowPhaseOrTable, true>), grid, dim3(kFftThreads), 0, s, a);
            else
                hipLaunchKernelGGL((k_fft_row4096_iono<kRowPhaseOrTable, false>), grid, dim3(kFftThreads), 0, s, a);
        } else {
            const int64_t blocks = ((int64_t)njobs + (1 << a.log2C) - 1) >> a.log2C;
            hipLaunchKernelGGL(k_fft_rows_iono, dim3((unsigned)blocks), dim3(kFftThreads), 0, s, a);
        }
        hipError_t e = hipGetLastError();
        if (prof)
            prof->end(s);
        if (e != hipSuccess)
            return e;
    }
    if (fwd_only)
        return hipSuccess;
    for (int i = d - 2; i >= 0; --i) {
        hipError_t e = strided(i, true);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Bluestein (chirp-z) pieces.  With w_m = exp(i pi m^2 / N) and kn = (k^2 + n^2 - (k - n)^2) / 2,
// DFT_N(x)_k = conj(w_k) (a (*) b)_k with a_n = x_n conj(w_n) and b_m = w_m for |m| < N, the
// convolution taken circularly at a power-of-two length M >= 2N - 1.  The inverse DFT of
// X_k H_k is (1/N) conj(DFT_N(conj(X H))), and conj(X_k H_k) conj(w_k) = conj(c_k H_k) when
// X_k = conj(w_k) c_k, so the second convolution's input is simply conj(c_k H_k).

// w_m, the argument reduced exactly: m^2 mod 2N in integers, then pi * (that / N).
__device__ __forceinline__ float2 chirp_w(int64_t m, int64_t N)
{
    const int64_t r = (m * m) % (2 * N);
    double sn, cs;
    sincospi((double)r / (double)N, &sn, &cs);
    return make_float2((float)cs, (float)sn);
}

// a = x conj(w) zero-padded to M; b = the chirp placed circularly (b_m = b_{M-m} = w_m, m < N).
// The chirp b is stored scaled by 2^-(log2(M) / 2), about 1/sqrt(M): its spectrum then has
// magnitude about 1 instead of sqrt(M), which keeps the convolutions' float32 intermediates
// (the transform of a times the chirp spectrum, then the inverse transform's sums) a factor
// sqrt(M) further from overflow.  The steps after each convolution undo the exact power of two.
__device__ __forceinline__ float chirp_scale_inv(int64_t M)
{
    return ldexpf(1.f, (63 - __clzll((unsigned long long)M)) / 2);
}

// One job per blockIdx.y.
__global__ void __launch_bounds__(256) k_bluestein_pre(const BluesteinJob *jobs, BluesteinJob inl, int64_t M)
{
    const BluesteinJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x, N = jb.n;
    if (m >= M)
        return;
    float2 av = make_float2(0.f, 0.f), bv = make_float2(0.f, 0.f);
    if (m < N) {
        const float2 w = chirp_w(m, N);
        const float2 v = gload(jb.x, m);
        av = make_float2(v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y);  // v conj(w)
        bv = w;
    } else if (M - m < N) {
        bv = chirp_w(M - m, N);
    }
    const float sb = 1.f / chirp_scale_inv(M);  // exact: a power of two
    gmem(jb.a)[m] = av;
    gmem(jb.a + M)[m] = make_float2(bv.x * sb, bv.y * sb);
}

// c (first convolution, in a) -> conj(c_k H_k) for k < N, zero above.  The forward DFT is
// X_k = conj(w_k) c_k and the second convolution starts from conj(Y_k) conj(w_k), Y_k = X_k H_k,
// which is conj(c_k H_k); with a correlation (Y_k = X_k conj(R_k) H_k) it is conj(c_k H_k) R_k.
__global__ void __launch_bounds__(256) k_bluestein_mid(const BluesteinJob *jobs, BluesteinJob inl, int64_t M)
{
    const BluesteinJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, N = jb.n;
    if (k >= M)
        return;
    float2 v = make_float2(0.f, 0.f);
    if (k < N) {
        const IonoJob ph{nullptr, nullptr, jb.phase, jb.carrier, jb.fs, nullptr};
        const float si = chirp_scale_inv(M);  // the convolution carries the chirp's scale
        const float2 c = gload(jb.a, k);
        const float2 h = cmul(make_float2(c.x * si, c.y * si), iono_phase(ph, k, N));
        v = make_float2(h.x, -h.y);
        if (jb.corr)
            v = cmul(v, gload(jb.corr, k));
    }
    gmem(jb.a)[k] = v;
}

// c (the convolution, in a) -> y_k = conj(w_k) c_k for k < N: the forward DFT alone.
__global__ void __launch_bounds__(256) k_bluestein_fwd_post(const BluesteinJob *jobs, BluesteinJob inl, int64_t M)
{
    const BluesteinJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, N = jb.n;
    if (k >= N)
        return;
    const float si = chirp_scale_inv(M);
    const float2 w = chirp_w(k, N), c = gload(jb.a, k);
    gmem(jb.y)[k] = make_float2((w.x * c.x + w.y * c.y) * si, (w.x * c.y - w.y * c.x) * si);  // conj(w) c
}

// f (second convolution, in a) -> y_n = w_n conj(f_n) / N.
__global__ void __launch_bounds__(256) k_bluestein_post(const BluesteinJob *jobs, BluesteinJob inl, int64_t M)
{
    const BluesteinJob jb = jobs ? gload(jobs, blockIdx.y) : inl;
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x, N = jb.n;
    if (n >= N)
        return;
    const float2 w = chirp_w(n, N), v = gload(jb.a, n);
    const float sc = (float)(1.0 / (double)N) * chirp_scale_inv(M);  // the chirp's scale undone exactly
    // w conj(v)
    gmem(jb.y)[n] = make_float2((w.x * v.x + w.y * v.y) * sc, (w.y * v.x - w.x * v.y) * sc);
}

}  // namespace

namespace {

// spec[i] = r[i] for i < n_rep, else 0: a replica zero-padded to the transform length.
__global__ void __launch_bounds__(256) k_pad(const float2 *__restrict__ r, int64_t n_rep, float2 *__restrict__ spec,
                                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        gmem(spec)[i] = i < n_rep ? gload(r, i) : make_float2(0.f, 0.f);
}

}  // namespace

hipError_t launch_pad(const float2 *r, int64_t n_rep, float2 *dst, int64_t n, hipStream_t s)
{
    if (n <= 0 || n_rep < 0 || n_rep > n || (n + 255) / 256 > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r, n_rep, dst, n);
    return hipGetLastError();
}

int64_t bluestein_m(int64_t n)
{
    int64_t m = 1;
    while (m < 2 * n - 1)
        m <<= 1;
    return m;
}

hipError_t launch_iono(const FftPlan &plan, const float2 *tw4096, const IonoJob *jobs_dev,
                       const IonoJob *job_inline, int njobs, hipStream_t s, Profiler *prof, int factor)
{
    return launch_fft_impl(plan, tw4096, jobs_dev, job_inline, njobs, false, factor, s, prof);
}

hipError_t launch_fft_forward(const FftPlan &plan, const float2 *tw4096, const IonoJob *jobs_dev,
                              const IonoJob *job_inline, int njobs, hipStream_t s, Profiler *prof)
{
    return launch_fft_impl(plan, tw4096, jobs_dev, job_inline, njobs, true, kRowPhaseOrTable, s, prof);
}

size_t bluestein_work_bytes(int64_t n) { return (size_t)bluestein_m(n) * 2 * sizeof(float2); }

hipError_t launch_iono_bluestein(const FftPlan &mplan, const float2 *tw4096, const BluesteinJob *jobs_dev,
                                 const IonoJob *ffts_dev, const BluesteinJob &inl, int njobs, int64_t max_n,
                                 hipStream_t s, Profiler *prof)
{
    const int64_t M = mplan.n;
    if (njobs <= 0)
        return hipSuccess;
    if (njobs > 65535 || max_n < 2 || bluestein_m(max_n) > M || (!jobs_dev && (njobs != 1 || !inl.a)) ||
        (jobs_dev && !ffts_dev))
        return hipErrorInvalidValue;
    const dim3 gm((unsigned)((M + 255) / 256), (unsigned)njobs), gn((unsigned)((max_n + 255) / 256), (unsigned)njobs);
    auto small = [&](auto kernel, dim3 grid, auto... extra) {
        if (prof)
            prof->begin(kKBluestein, s);
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, s, jobs_dev, inl, extra...);
        const hipError_t e = hipGetLastError();
        if (prof)
            prof->end(s);
        return e;
    };
    hipError_t e = small(k_bluestein_pre, gm, M);
    if (e != hipSuccess)
        return e;
    // the chirp spectra, in the native bin order the convolutions multiply in
    const IonoJob jb_b{inl.a + M, inl.a + M, PhaseNum{}, 0.0, 0.0, nullptr};
    const IonoJob conv{inl.a, inl.a, PhaseNum{}, 0.0, 0.0, inl.a + M};
    const IonoJob *fb = jobs_dev ? ffts_dev : nullptr, *fc = jobs_dev ? ffts_dev + njobs : nullptr;
    e = launch_fft_forward(mplan, tw4096, fb, &jb_b, njobs, s, prof);
    if (e == hipSuccess)
        e = launch_iono(mplan, tw4096, fc, &conv, njobs, s, prof);
    if (e == hipSuccess)
        e = small(k_bluestein_mid, gm, M);
    if (e == hipSuccess)
        e = launch_iono(mplan, tw4096, fc, &conv, njobs, s, prof);
    if (e == hipSuccess)
        e = small(k_bluestein_post, gn, M);
    return e;
}

hipError_t launch_bluestein_forward(const FftPlan &mplan, const float2 *tw4096, const BluesteinJob &inl,
                                    hipStream_t s, Profiler *prof)
{
    const int64_t M = mplan.n;
    if (inl.n < 2 || bluestein_m(inl.n) > M || !inl.a)
        return hipErrorInvalidValue;
    const dim3 gm((unsigned)((M + 255) / 256)), gn((unsigned)((inl.n + 255) / 256));
    const BluesteinJob *none = nullptr;
    if (prof)
        prof->begin(kKBluestein, s);
    hipLaunchKernelGGL(k_bluestein_pre, gm, dim3(256), 0, s, none, inl, M);
    hipError_t e = hipGetLastError();
    if (prof)
        prof->end(s);
    const IonoJob jb_b{inl.a + M, inl.a + M, PhaseNum{}, 0.0, 0.0, nullptr};
    const IonoJob conv{inl.a, inl.a, PhaseNum{}, 0.0, 0.0, inl.a + M};
    if (e == hipSuccess)
        e = launch_fft_forward(mplan, tw4096, nullptr, &jb_b, 1, s, prof);
    if (e == hipSuccess)
        e = launch_iono(mplan, tw4096, nullptr, &conv, 1, s, prof);
    if (e != hipSuccess)
        return e;
    if (prof)
        prof->begin(kKBluestein, s);
    hipLaunchKernelGGL(k_bluestein_fwd_post, gn, dim3(256), 0, s, none, inl, M);
    e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace rc
