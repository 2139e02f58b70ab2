// sinc_mfma.hip -- the windowed-sinc tap sum of Eq (17) (Kaiser taper, Sec. III-B) as a
// matrix product on the gfx950 matrix cores.
//
// A 2048-output workgroup tile shares one integer shift S: output m of the tile sits at
// t = alpha m = m + S + sigma_m with sigma_m = sigma_c + eps (m - m_c), eps = alpha - 1, and
// |sigma_m - sigma_c| <= |eps| * 1023.5 <= 0.0614 for |eps| <= 6e-5.  Its tap weights
// h(sigma_m - k), k = -H .. H, are taken from a quartic in z = (sigma_m - sigma_p) / delta_max
// around the nearest point sigma_p = p / 128 of a phase grid (|z| <= 1, delta_max = 0.0654):
//     h(sigma_p + delta_max z - k) ~= sum_r a_{p,r}[k] z^r,
// interpolated in float64 at five Chebyshev nodes (tap error ~3e-8).  The 129 grid phases are
// tabulated once per (H, beta) by k_sinc_table, already split into fp16 hi/lo and laid out as
// matrix-core B fragments.  Then
//     y[m] = sum_r z_m^r Z_r[m],   Z_r[m] = sum_k x[m + S + k] a_{p,r}[k],
// and for a 256-output sub-tile m = m0 + 16 i + u the contraction is a GEMM
//     Z_r[i][u] = sum_kappa X[i][kappa] B_r[kappa][u],
//     X[i][kappa] = x[m0 + 16 i + S - H + kappa]   (Hankel: 8-sample aligned runs per lane),
//     B_r[kappa][u] = a_{p,r}[kappa - u - H]        (the column shift u lives in B).
// kappa runs over 2H + 16 taps rounded up to whole 32-wide MFMA steps.  Both operands are split
// into float16 hi + lo parts after exact power-of-two scaling.  Orders 0 and 1 accumulate
// hi*hi + hi*lo + lo*hi in float32 (v_mfma_f32_16x16x32_f16, about 22 bits per product); the
// higher orders, whose terms are at most a few parts in 1e3 of the output for band-limited
// input, take hi*hi alone (11 bits).
//
// Batches of many tiles run persistent workgroups over a tile list sorted by phase (built on the
// device by k_mf_tile_phase, k_mf_tile_count and k_mf_tile_scatter): a workgroup walks a run of
// that list, copies a phase's B block into LDS only when the phase changes, and prefetches the
// next tile's input into registers while the matrix cores work on the current one.  Consecutive
// workgroup indices are spread over the eight XCDs, so each XCD's L2 serves a contiguous range of
// phases.  Each wave stages its own part of the tile's input (two sub-tiles at H = 64, one at
// H = 128, so that a SIMD always runs two waves) into LDS with its own scale, in a bank swizzle
// that keeps the Hankel fragment reads free of conflicts.
#include <cmath>
#include <vector>

#include "rc_internal.h"

namespace rc {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// two float32 values to a pair of float16, rounded toward zero (v_cvt_pkrtz_f16_f32)
__device__ __forceinline__ half2v pkrtz(float a, float b)
{
    return __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(a, b));
}

constexpr int kMfOut = kSincMfmaTile;  // outputs per tile (one phase-grid point)
constexpr int kSubTile = 256;          // outputs of one 16 x 16 matrix-core product
constexpr int kMfOrders = 5;           // quartic in the drift
constexpr int kMfLo = 2;               // orders that also take the hi*lo and lo*hi products
constexpr int kMfBlk = kMfOrders + kMfLo;  // 1 KiB B fragments per 32-tap step
constexpr int kXcds = 8;               // workgroups are dealt round-robin to this many XCDs
constexpr int kCoefExp = 12;           // coefficients are scaled by 2^12 before the fp16 split
constexpr double kMfHalf = 0.5 * (kMfOut - 1);  // 1023.5: half-width of the tile in outputs
constexpr int kPhases = 128;                    // phase grid points per sample
constexpr int kPhaseRows = kPhases + 1;         // sigma_p = p / 128, p = -64 .. 64
constexpr double kDeltaMax = 0.0654;            // >= 6e-5 * 1023.5 + 1 / 256

template <int H>
struct MfGeom {
    static constexpr int ntap = 2 * H + 1;
    static constexpr int kext = ((2 * H + 16) + 31) / 32 * 32;
    static constexpr int ksteps = kext / 32;
    // Sub-tiles per wave: two at H = 64, whose LDS fits two four-wave workgroups per CU; one at
    // H = 128, where a four-wave workgroup would be alone on its CU with one wave per SIMD, so
    // the tile goes to eight waves sharing one B block (two waves per SIMD).
    static constexpr int nsub = H <= 64 ? 2 : 1;
    static constexpr int nwaves = kSincMfmaTile / (nsub * kSubTile);
    static constexpr int threads = 64 * nwaves;
    static constexpr int wout = nsub * kSubTile;               // outputs per wave and tile
    static constexpr int wspan = wout + kext;                  // samples staged per wave
    static constexpr int wpp = (wspan + 127) / 128;            // staged sample pairs per lane
    static constexpr int rowlen = kext + 32;                   // padded coefficient row (halves)
    static constexpr int node_iters = (ntap + 47) / 48;       // 12 taps x 5 nodes per wave
    static constexpr int bbytes = ksteps * kMfBlk * 1024;  // B fragments of one phase
    // main kernel LDS: B block, then per wave 4 fp16 arrays of `wspan` (re hi, re lo, im hi,
    // im lo; 64-byte multiples, so every region stays 16-byte aligned), sample e at a_pad(e)
    static constexpr int a_off = bbytes;
    static constexpr int pspan = wspan;                        // halves per array
    static constexpr int a_wave = 4 * pspan;                   // halves per wave region
    static constexpr int bytes = a_off + nwaves * a_wave * 2;
    // table kernel LDS: coefficient rows [order][part][rowlen]
    static constexpr int rows_bytes = kMfOrders * 2 * rowlen * 2;
};

static_assert(MfGeom<64>::nwaves * MfGeom<64>::wout == kMfOut && MfGeom<128>::nwaves * MfGeom<128>::wout == kMfOut,
              "the waves' sub-tiles cover a tile");
static_assert(MfGeom<64>::wspan % 32 == 0 && MfGeom<128>::wspan % 32 == 0, "wave regions stay aligned");

// Position of span sample e in a staged array.  A fragment read serves eight lanes of a row at a
// time, 16 bytes each at 32-byte steps, against 128 bytes of banks: lanes i and i + 4 would hit
// the same banks.  Swapping the two 16-byte halves of every other 128 bytes separates them.
// Runs of 8 samples that start at a multiple of 8 stay contiguous, and
// a_pad(e + 256) = a_pad(e) + 256.
__device__ __forceinline__ int a_pad(int e) { return e ^ (((e >> 6) & 1) << 3); }

// The Kaiser series with a fixed number of terms NT >= kp.n (terms past kp.n are zero).
constexpr int kMfKaiserTerms = 32;

template <int NT>
__device__ __forceinline__ double kaiser_at_m(const KaiserPoly &kp, double x)
{
    const double s = 1.0 - x * x;
    double acc = kp.c[NT - 1];
#pragma unroll
    for (int j = NT - 2; j >= 0; --j)
        acc = fma(acc, s, kp.c[j]);
    return acc;
}

// One workgroup per grid phase p: the quartic of every tap (float64 at the five Chebyshev
// nodes of [-delta_max, delta_max]), split into fp16 hi/lo, arranged as B fragments: step s
// holds the hi blocks of orders 0..4, then the lo blocks of orders 0..kMfLo-1; a block holds,
// for lane l, the 8 halves B_r[32 s + 8 (l / 16) + j][l % 16].
template <int H, int NT>
__global__ void __launch_bounds__(256) k_sinc_table(KaiserPoly kp, MfmaSincConst mc, unsigned char *table)
{
    using G = MfGeom<H>;
    __shared__ unsigned short rows[G::rows_bytes / 2];  // fp16 bit patterns, row pos 16 + t = tap t
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double sp = (double)((int)blockIdx.x - kPhases / 2) / kPhases;
    const int grp = lane / 5, node = lane - 5 * grp;
    const bool active = grp < 12;
    const int nd = active ? node : 0;
    const double un = sp + kDeltaMax * mc.node[nd];  // node position relative to tap 0
    const double sn = sinpi(un);
    const float cscale = ldexpf(1.0f, kCoefExp);
    for (int it = 0; it < G::node_iters; ++it) {
        const int t = 48 * it + 12 * wave + grp;
        const int k = t - H;
        double h = 0.0;
        const double u = un - (double)k;
        if (active && t < G::ntap && fabs(u) < (double)H) {
            const double sgn = (k & 1) ? -sn : sn;
            h = (u == 0.0 ? 1.0 : sgn / (kPi * u)) * kaiser_at_m<NT>(kp, u / (double)H);
        }
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < kMfOrders; ++i)
            a = fma(mc.vinv[nd * kMfOrders + i], __shfl(h, active ? 5 * grp + i : lane, 64), a);
        if (active && t < G::ntap) {
            const float c = (float)a * cscale;
            const _Float16 ch = (_Float16)c;
            const _Float16 cl = (_Float16)(c - (float)ch);
            rows[(node * 2 + 0) * G::rowlen + 16 + t] = __builtin_bit_cast(unsigned short, ch);
            rows[(node * 2 + 1) * G::rowlen + 16 + t] = __builtin_bit_cast(unsigned short, cl);
        }
    }
    for (int p = tid; p < kMfOrders * 2 * G::rowlen; p += 256) {
        const int pos = p % G::rowlen;
        if (pos < 16 || pos >= 16 + G::ntap)
            rows[p] = 0;
    }
    __syncthreads();
    unsigned char *out = table + (size_t)blockIdx.x * G::bbytes;
    for (int id = tid; id < G::ksteps * kMfBlk * 64; id += 256) {
        const int l = id & 63, blk = id >> 6;  // blk = s * kMfBlk + j
        const int s = blk / kMfBlk, j = blk - s * kMfBlk;
        const int part = j < kMfOrders ? 0 : 1, r = j < kMfOrders ? j : j - kMfOrders;
        const int u = l & 15;
        const int o = 16 + 32 * s + 8 * (l >> 4) - u;  // first half of the fragment in the row
        uint4 f;
        unsigned w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            w[j] = (unsigned)rows[(r * 2 + part) * G::rowlen + o + 2 * j] |
                   ((unsigned)rows[(r * 2 + part) * G::rowlen + o + 2 * j + 1] << 16);
        f.x = w[0];
        f.y = w[1];
        f.z = w[2];
        f.w = w[3];
        reinterpret_cast<uint4 *>(out + blk * 1024)[l] = f;
    }
}

// Where a tile of outputs M0 .. M0 + 2047 sits in the input: shift S, offset sigma_c of its
// centre from sample M0 + 1023.5 + S, and the nearest grid phase p / 128.
struct MfTile {
    double Sd;  // S as a double
    double sc;  // sigma at the tile centre, in [-1/2, 1/2]
    int p;      // grid phase, -64 .. 64
};

__device__ __forceinline__ MfTile mf_tile(double alpha, int64_t M0)
{
    const double eps = alpha - 1.0;
    const double mcen = (double)M0 + kMfHalf;
    MfTile t;
    t.Sd = rint(eps * mcen);
    t.sc = eps * mcen - t.Sd;
    int p = (int)rint(t.sc * kPhases);
    t.p = p < -kPhases / 2 ? -kPhases / 2 : (p > kPhases / 2 ? kPhases / 2 : p);
    return t;
}

// Tile list, step 1: every (job, tile) writes its reference and its phase at its flat index
// tile0 + tile.  Grid: (tile blocks of 256, jobs).
__global__ void __launch_bounds__(256)
k_mf_tile_phase(const SincJob *__restrict__ jobs, uint2 *__restrict__ ref, unsigned char *__restrict__ phase)
{
    const SincJob jb = gload(jobs, blockIdx.y);
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t * kMfOut >= jb.n_out)
        return;
    const MfTile tp = mf_tile(jb.alpha, t * kMfOut);
    ref[jb.tile0 + t] = make_uint2(blockIdx.y, (unsigned)t);
    phase[jb.tile0 + t] = (unsigned char)(tp.p + kPhases / 2);
}

// Tile list, steps 2 and 3: a counting sort of the references by phase over chunks of
// kSortChunk tiles, one workgroup per chunk.  Step 2 counts each chunk's phases; step 3 turns
// the counts of all chunks into the chunk's first slot per phase and scatters.  The order of
// equal phases is arbitrary; no output depends on it.
constexpr int kSortChunk = 256;

__global__ void __launch_bounds__(256)
k_mf_tile_count(const unsigned char *__restrict__ phase, int64_t ntiles, unsigned *__restrict__ counts)
{
    __shared__ unsigned cnt[kPhaseRows];
    const int tid = threadIdx.x;
    if (tid < kPhaseRows)
        cnt[tid] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kSortChunk;
    const int64_t i1 = i0 + kSortChunk < ntiles ? i0 + kSortChunk : ntiles;
    for (int64_t i = i0 + tid; i < i1; i += 256)
        atomicAdd(&cnt[phase[i]], 1u);
    __syncthreads();
    if (tid < kPhaseRows)
        counts[(size_t)blockIdx.x * kPhaseRows + tid] = cnt[tid];
}

__global__ void __launch_bounds__(256)
k_mf_tile_scatter(const uint2 *__restrict__ ref, const unsigned char *__restrict__ phase, int64_t ntiles,
                  const unsigned *__restrict__ counts, uint2 *__restrict__ list)
{
    __shared__ unsigned tot[kPhaseRows], base[kPhaseRows];
    const int tid = threadIdx.x;
    const int nchunks = gridDim.x, me = blockIdx.x;
    if (tid < kPhaseRows) {
        // eight chunks' counts in flight at a time
        unsigned all = 0, before = 0;
        for (int w0 = 0; w0 < nchunks; w0 += 8) {
            unsigned c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                c[u] = w0 + u < nchunks ? counts[(size_t)(w0 + u) * kPhaseRows + tid] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                all += c[u];
                before += w0 + u < me ? c[u] : 0u;
            }
        }
        tot[tid] = all;
        base[tid] = before;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned run = 0;
        for (int p = 0; p < kPhaseRows; ++p) {
            base[p] += run;
            run += tot[p];
        }
    }
    __syncthreads();
    const int64_t i0 = (int64_t)me * kSortChunk;
    const int64_t i1 = i0 + kSortChunk < ntiles ? i0 + kSortChunk : ntiles;
    for (int64_t i = i0 + tid; i < i1; i += 256)
        list[atomicAdd(&base[phase[i]], 1u)] = ref[i];
}

// The resampling GEMM.  Without a list, workgroup (x, y) computes tile x of job y.  With a list,
// the grid is persistent: workgroup b takes the run c(b) of the sorted list, where c deals
// consecutive b to different XCDs so that an XCD holds a contiguous range of phases.
//
// Wave w owns outputs wout w .. wout (w + 1) - 1 of the workgroup's tile (its nsub sub-tiles of
// 256) and stages the input they read, wspan = wout + kext samples, into an LDS region of its
// own with a scale of its own: the waves share only the phase's B block.
// A tile of the persistent loop: its job, first output and position in the input.
struct MfCur {
    SincJob jb;
    int64_t M0;
    MfTile tp;
};

// Largest of a non-negative float over the wave, uniform: the bit patterns of non-negative
// floats order like their values, so the maximum is taken on them, within each row of 16 lanes
// by DPP moves (quad permutations, then rotations by 4 and 8), then over the rows' first lanes.
__device__ __forceinline__ float wave_max_nonneg(float v)
{
    int u = __float_as_int(v);
    u = max(u, __builtin_amdgcn_update_dpp(0, u, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    u = max(u, __builtin_amdgcn_update_dpp(0, u, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    u = max(u, __builtin_amdgcn_update_dpp(0, u, 0x124, 0xF, 0xF, false));  // row_ror:4
    u = max(u, __builtin_amdgcn_update_dpp(0, u, 0x128, 0xF, 0xF, false));  // row_ror:8
    const int a = max(__builtin_amdgcn_readlane(u, 0), __builtin_amdgcn_readlane(u, 16));
    const int b = max(__builtin_amdgcn_readlane(u, 32), __builtin_amdgcn_readlane(u, 48));
    return __int_as_float(max(a, b));
}

// max(m, |a|, |b|) in one instruction: v_max3_f32 with absolute-value source modifiers.  fmaxf
// on loaded samples, which the compiler cannot prove canonical, would first quiet each of them
// with an instruction of its own.  A quiet NaN operand is ignored either way; signalling NaNs do
// not come out of arithmetic.
__device__ __forceinline__ float max3_abs(float m, float a, float b)
{
    float r;
    asm("v_max3_f32 %0, %1, |%2|, |%3|" : "=v"(r) : "v"(m), "v"(a), "v"(b));
    return r;
}

// A wave-uniform 64-bit integer held in scalar registers (the value of the first active lane).
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Orders memory operations of one wave on LDS: what its lanes stored before is what its lanes
// load after.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile i of the sorted list.
__device__ __forceinline__ MfCur mf_list_tile(const SincJob *__restrict__ jobs, const uint2 *__restrict__ list,
                                              int64_t i)
{
    const uint2 e = gload(list, i);
    MfCur t;
    t.jb = gload(jobs, e.x);
    t.M0 = (int64_t)e.y * kMfOut;
    t.tp = mf_tile(t.jb.alpha, t.M0);
    return t;
}

// Phase p's B fragments into LDS, by the whole workgroup (NT threads), four 16-byte loads in
// flight per thread; the caller brackets it with barriers.  Indices past the block are clamped
// to its last element, which is then copied more than once with the same value: no branches,
// so every load is complete when the copy ends.
template <int H, int NT>
__device__ __forceinline__ void mf_load_b(const unsigned char *__restrict__ table, int p, unsigned char *bsm,
                                          int tid)
{
    using G = MfGeom<H>;
    const auto src = gmem(reinterpret_cast<const uint4 *>(table + (size_t)(p + kPhases / 2) * G::bbytes));
    uint4 *dst = reinterpret_cast<uint4 *>(bsm);
    constexpr int n16 = G::bbytes / 16;
#pragma unroll 1
    for (int k = tid; k < n16; k += 4 * NT) {
        const int k1 = k + NT < n16 ? k + NT : n16 - 1;
        const int k2 = k + 2 * NT < n16 ? k + 2 * NT : n16 - 1;
        const int k3 = k + 3 * NT < n16 ? k + 3 * NT : n16 - 1;
        const uint4 v0 = src[k], v1 = src[k1], v2 = src[k2], v3 = src[k3];
        dst[k] = v0;
        dst[k1] = v1;
        dst[k2] = v2;
        dst[k3] = v3;
    }
}

// One wave's part of a tile: the fetch of its input span into registers, the staging into its
// LDS region, the matrix products and the stores.
template <int H>
struct MfWave {
    using G = MfGeom<H>;
    const unsigned char *bsm;        // the phase's B block
    _Float16 *a_rh, *a_rl, *a_ih, *a_il;  // this wave's region: re hi, re lo, im hi, im lo
    int lane, wbase;                 // wbase: this wave's first output in a tile
    float2 xv[G::wpp][2];            // the fetched span, two samples per lane and step
    floatx4 acc[G::nsub][kMfOrders][2];  // Z_r of the wave's sub-tiles, re and im

    __device__ __forceinline__ MfWave(unsigned char *smem, int region, int lane_, int wbase_)
        : bsm(smem), lane(lane_), wbase(wbase_)
    {
        a_rh = reinterpret_cast<_Float16 *>(smem + G::a_off) + region * G::a_wave;
        a_rl = a_rh + G::pspan;
        a_ih = a_rl + G::pspan;
        a_il = a_ih + G::pspan;
    }

    // this wave has outputs in tile t (uniform over the wave)
    __device__ __forceinline__ bool active(const MfCur &t) const { return t.M0 + wbase < t.jb.n_out; }

    // samples lo .. lo + wspan - 1 of the input, two per lane and step
    __device__ __forceinline__ void fetch(const MfCur &t)
    {
        const int64_t lo = uniform64(t.M0 + (int64_t)t.tp.Sd - H + wbase);
        if (lo >= 0 && lo + G::wspan <= t.jb.n_in) {
            // the whole span lies inside x (the usual case; uniform): 32-bit offsets from its start
            const auto xs = gmem(t.jb.x) + lo;
#pragma unroll
            for (int q = 0; q < G::wpp; ++q) {
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int e = 2 * lane + 128 * q + h2;
                    const float2 v = xs[e < G::wspan ? e : G::wspan - 1];
                    xv[q][h2] = e < G::wspan ? v : make_float2(0.f, 0.f);
                }
            }
            return;
        }
        const int64_t last = t.jb.n_in - 1;
        const auto xs = gmem(t.jb.x);
        // every lane loads an in-bounds sample (index clamped) and zeroes what lies outside x
        // or past the span: no branch between the loads
#pragma unroll
        for (int q = 0; q < G::wpp; ++q) {
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int e = 2 * lane + 128 * q + h2;
                const int64_t g = lo + e;
                const bool ok = e < G::wspan && g >= 0 && g <= last;
                const int64_t gc = g < 0 ? 0 : (g > last ? last : g);
                const float2 v = xs[gc];
                xv[q][h2] = ok ? v : make_float2(0.f, 0.f);
            }
        }
    }

    // The fetched span into this wave's region, scaled by a power of two (largest component in
    // [2^10, 2^11)) and split into fp16 hi/lo; returns the scale exponent.
    __device__ __forceinline__ int stage()
    {
        float mx = 0.f;
#pragma unroll
        for (int q = 0; q < G::wpp; ++q)
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
                mx = max3_abs(mx, xv[q][h2].x, xv[q][h2].y);
        mx = wave_max_nonneg(mx);
        int xe = 0;
        if (mx > 0.f) {
            int E;
            frexpf(mx, &E);  // mx = f 2^E, f in [0.5, 1)
            xe = 11 - E;
        }
        const float xs2 = ldexpf(1.0f, xe);
        wave_lds_sync();  // this wave's loads of the previous tile's operands come first
#pragma unroll
        for (int q = 0; q < G::wpp; ++q) {
            const int e = 2 * lane + 128 * q;
            if (e < G::wspan) {  // wspan is even: a pair is either wholly inside or outside
                // hi rounds toward zero (one packed conversion per pair); the residual x - hi is
                // exact in float32 and becomes lo
                const float r0 = xv[q][0].x * xs2, r1 = xv[q][1].x * xs2;
                const float i0f = xv[q][0].y * xs2, i1f = xv[q][1].y * xs2;
                const half2v rh = pkrtz(r0, r1);
                const half2v ih = pkrtz(i0f, i1f);
                const half2v rl = pkrtz(r0 - (float)rh[0], r1 - (float)rh[1]);
                const half2v il = pkrtz(i0f - (float)ih[0], i1f - (float)ih[1]);
                const int pe = a_pad(e);
                *reinterpret_cast<half2v *>(a_rh + pe) = rh;
                *reinterpret_cast<half2v *>(a_rl + pe) = rl;
                *reinterpret_cast<half2v *>(a_ih + pe) = ih;
                *reinterpret_cast<half2v *>(a_il + pe) = il;
            }
        }
        wave_lds_sync();  // and its lanes' stores are seen by its lanes' fragment loads
        return xe;
    }

    // The matrix products of the staged span with the B block.  The wave runs its sub-tiles
    // together: each B fragment is read from LDS once per 32-tap step for all of them.  A fragments:
    // lane (i, q) = (l % 16, l / 16) holds the 8 samples at 16 i + 8 q + 32 s of its sub-tile's
    // span (aligned 8-sample runs of the Hankel matrix).
    //
    // A step runs, sub-tile by sub-tile, three groups of products: lo*hi of the low orders (xl,
    // bh), hi*hi of every order (xh, bh), hi*lo of the low orders (xh, bl).  Each register of
    // the step's fragments is refilled with the next step's as soon as its last product of this
    // step has issued: a sub-tile's xl after its first group and its xh[c] after its hi*lo
    // products, bh[r] after the last sub-tile's hi*hi products of order r, bl last.  With two
    // sub-tiles every fragment has at least twelve products to hide its read behind (four with
    // one).  Scheduling barriers keep the compiler from moving the reads next to their first use.
    __device__ __forceinline__ void gemm()
    {
        const int arow = 16 * (lane & 15) + 8 * (lane >> 4);
        half8 xh[G::nsub][2], xl[G::nsub][2], bh[kMfOrders], bl[kMfLo];  // x: [sub-tile][re/im]
        const _Float16 *const xre[2] = {a_rh, a_rl}, *const xim[2] = {a_ih, a_il};
        auto ld_x = [&](int lo, int s, int t, int c2) {
            const _Float16 *const base = c2 ? xim[lo] : xre[lo];
            return *reinterpret_cast<const half8 *>(base + a_pad(arow + 32 * s) + kSubTile * t);
        };
        auto ld_b = [&](int s, int j) {
            return reinterpret_cast<const half8 *>(bsm + s * kMfBlk * 1024)[64 * j + lane];
        };
        auto mfma = [&](const half8 &x, const half8 &w, floatx4 &c, bool zero) {
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, w, zero ? floatx4{0.f, 0.f, 0.f, 0.f} : c, 0, 0, 0);
        };
        // step s; the first starts every accumulator from zero (the matrix core's inline
        // constant), so nothing is cleared beforehand; `more`: read step s + 1's fragments
        auto kstep = [&](int s, bool first, bool more) {
#pragma unroll
            for (int t = 0; t < G::nsub; ++t) {
                const bool last = t == G::nsub - 1;
#pragma unroll
                for (int r = 0; r < kMfLo; ++r)
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2)
                        mfma(xl[t][c2], bh[r], acc[t][r][c2], first);
                __builtin_amdgcn_sched_barrier(0);
                if (more) {
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2)
                        xl[t][c2] = ld_x(1, s + 1, t, c2);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < kMfOrders; ++r) {
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2)
                        mfma(xh[t][c2], bh[r], acc[t][r][c2], first && r >= kMfLo);
                    if (last) {
                        __builtin_amdgcn_sched_barrier(0);
                        if (more)
                            bh[r] = ld_b(s + 1, r);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
#pragma unroll
                for (int c2 = 0; c2 < 2; ++c2) {
#pragma unroll
                    for (int r = 0; r < kMfLo; ++r)
                        mfma(xh[t][c2], bl[r], acc[t][r][c2], false);
                    __builtin_amdgcn_sched_barrier(0);
                    if (more)
                        xh[t][c2] = ld_x(0, s + 1, t, c2);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (more) {
#pragma unroll
                for (int r = 0; r < kMfLo; ++r)
                    bl[r] = ld_b(s + 1, kMfOrders + r);
            }
            __builtin_amdgcn_sched_barrier(0);
        };
#pragma unroll
        for (int t = 0; t < G::nsub; ++t)
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
                xl[t][c2] = ld_x(1, 0, t, c2);
#pragma unroll
        for (int r = 0; r < kMfOrders; ++r)
            bh[r] = ld_b(0, r);
#pragma unroll
        for (int t = 0; t < G::nsub; ++t)
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
                xh[t][c2] = ld_x(0, 0, t, c2);
#pragma unroll
        for (int r = 0; r < kMfLo; ++r)
            bl[r] = ld_b(0, kMfOrders + r);
        kstep(0, true, true);
#pragma unroll 1
        for (int s = 1; s < G::ksteps - 1; ++s)
            kstep(s, false, true);
        kstep(G::ksteps - 1, false, false);
    }

    // Lane holds Z_r[row 4 (l/16) + j][col l % 16] of each sub-tile: output
    // m = M0 + wbase + 256 t + 16 row + col.  z is linear in m.  Outputs next to an exact sample
    // instant (sigma within 1e-5 of 0), where alpha m may round to an integer, are checked in
    // float64 and, if exact, rewritten with the input sample after all stores are issued (a load
    // between the stores would make each store wait).
    __device__ __forceinline__ void store(const MfCur &c, int xe)
    {
        const double alpha = c.jb.alpha, eps = alpha - 1.0;
        const int64_t S = (int64_t)c.tp.Sd;
        const float unscale = ldexpf(1.0f, -(xe + kCoefExp));
        // z_m = (sigma_m - sigma_p) / delta_max = z_c + (m - mcen) eps / delta_max
        const float zc = (float)((c.tp.sc - (double)c.tp.p * (1.0 / kPhases)) * (1.0 / kDeltaMax));
        const float zstep = (float)(eps * (1.0 / kDeltaMax));
        const float sc32 = (float)c.tp.sc;
        const float e32 = (float)eps;
        const auto yt = gmem(c.jb.y) + c.M0;  // this tile's first output
        const bool full = c.M0 + kMfOut <= c.jb.n_out;  // uniform
        const int nvalid = full ? kMfOut : (int)(c.jb.n_out - c.M0);
        // sigma runs over sc +- |eps| 1023.5 in this tile: only if that range comes within 1e-5
        // of 0 can an output sit on an exact sample instant (uniform)
        const bool may_hit = fabs(c.tp.sc) <= fabs(eps) * kMfHalf + 2e-5;
        // output (t, j) of this lane is m - M0 = loff + 256 t + 16 j
        const int loff = wbase + 64 * (lane >> 4) + (lane & 15);
        const float dml = (float)loff - (float)kMfHalf;  // m - mcen, exact like every sum below
        auto poly = [&](int t, int j, float z) {
            float yr = acc[t][kMfOrders - 1][0][j], yi = acc[t][kMfOrders - 1][1][j];
#pragma unroll
            for (int r = kMfOrders - 2; r >= 0; --r) {
                yr = fmaf(yr, z, acc[t][r][0][j]);
                yi = fmaf(yi, z, acc[t][r][1][j]);
            }
            return make_float2(yr * unscale, yi * unscale);
        };
        float2 *const yl = c.jb.y + c.M0 + loff;
        unsigned near = 0;  // bit 4 t + j: output (t, j) is next to an exact instant
        if (full && !may_hit) {
            // the usual tile (uniform): no output to check, constant offsets from the lane's first
#pragma unroll
            for (int t = 0; t < G::nsub; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float dm = dml + (float)(kSubTile * t + 16 * j);
                    store_nt(yl + kSubTile * t + 16 * j, poly(t, j, fmaf(dm, zstep, zc)));
                }
        } else {
#pragma unroll
            for (int t = 0; t < G::nsub; ++t) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (!full && loff + kSubTile * t + 16 * j >= nvalid)
                        continue;
                    const float dm = dml + (float)(kSubTile * t + 16 * j);
                    if (may_hit && fabsf(fmaf(dm, e32, sc32)) < 1e-5f)
                        near |= 1u << (4 * t + j);
                    store_nt(yl + kSubTile * t + 16 * j, poly(t, j, fmaf(dm, zstep, zc)));
                }
            }
        }
        if (__any(near != 0)) {  // rare: uniform over the wave
            const auto xg = gmem(c.jb.x);
#pragma unroll 1
            for (int b = 0; b < 4 * G::nsub; ++b) {
                if (!((near >> b) & 1u))
                    continue;
                const int t = b >> 2, j = b & 3;
                const int off = loff + kSubTile * t + 16 * j;
                const int64_t m = c.M0 + off;
                const double md = (double)m;
                if (((__dmul_rn(alpha, md) - md) - c.tp.Sd) == 0.0) {
                    const int64_t src = m + S;
                    float2 v = make_float2(0.f, 0.f);
                    if (src >= 0 && src < c.jb.n_in)
                        v = xg[src];
                    yt[off] = v;
                }
            }
        }
    }
};

// One tile at a time (four waves of two sub-tiles at H = 64, eight of one at H = 128): the tiles
// of a list run (persistent grid), or without a list tile blockIdx.x of job blockIdx.y.  Per
// tile: the matrix products, then the staging of the next tile's span (its loads were issued a
// tile ahead, before this wave's previous stores) and the fetch of the one after, then this
// tile's stores.  The waves wait for each other only when the phase changes.  Two workgroups
// share a CU at H = 64, one at H = 128 (LDS); either way a SIMD runs two waves.
template <int H>
constexpr int mf_wg_per_cu() { return 2 * MfGeom<H>::bytes <= 160 * 1024 ? 2 : 1; }

template <int H>
__global__ void __launch_bounds__(MfGeom<H>::threads, mf_wg_per_cu<H>())
k_sinc_mfma(const SincJob *__restrict__ jobs, SincJob inl, const uint2 *__restrict__ list, int64_t ntiles,
            const unsigned char *__restrict__ table)
{
    using G = MfGeom<H>;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    MfWave<H> W(smem, wave, lane, G::wout * wave);

    int64_t i0 = 0, i1 = 1;
    if (list) {
        const int64_t g = gridDim.x, b = blockIdx.x;
        const int64_t c = g % kXcds == 0 ? (b % kXcds) * (g / kXcds) + b / kXcds : b;
        i0 = c * ntiles / g;
        i1 = (c + 1) * ntiles / g;
        if (i0 >= i1)
            return;  // uniform over the workgroup
    }
    auto tile_at = [&](int64_t i) {
        if (list)
            return mf_list_tile(jobs, list, i);
        MfCur t;
        t.jb = jobs ? gload(jobs, blockIdx.y) : inl;
        t.M0 = (int64_t)blockIdx.x * kMfOut;
        t.tp = mf_tile(t.jb.alpha, t.M0);
        return t;
    };

    MfCur cur = tile_at(i0);
    if (cur.M0 >= cur.jb.n_out)
        return;  // only without a list (ragged jobs); uniform over the workgroup
    int cur_p = cur.tp.p;
    mf_load_b<H, G::threads>(table, cur_p, smem, tid);
    if (W.active(cur))
        W.fetch(cur);
    int xe = W.active(cur) ? W.stage() : 0;
    MfCur nxt = cur;
    if (i0 + 1 < i1) {
        nxt = tile_at(i0 + 1);
        if (W.active(nxt))
            W.fetch(nxt);
    }
    __syncthreads();  // the first phase's B block is in LDS

    for (int64_t i = i0; i < i1; ++i) {
        if (cur.tp.p != cur_p) {  // uniform over the workgroup: every wave walks the same run
            __syncthreads();      // every wave is done with the previous block
            mf_load_b<H, G::threads>(table, cur.tp.p, smem, tid);
            cur_p = cur.tp.p;
            __syncthreads();
        }
        const MfCur c = cur;
        const int cxe = xe;
        const bool active = W.active(c);
        if (active) {
            // the products at the highest issue priority: when the other wave on this SIMD is in
            // its vector phase, the matrix core's next instruction still issues first
            __builtin_amdgcn_s_setprio(3);
            W.gemm();
            __builtin_amdgcn_s_setprio(0);
        }
        if (i + 1 < i1) {
            cur = nxt;
            xe = W.active(cur) ? W.stage() : 0;
            if (i + 2 < i1) {
                nxt = tile_at(i + 2);
                if (W.active(nxt))
                    W.fetch(nxt);
            }
        }
        if (active)
            W.store(c, cxe);
    }
}

// Chebyshev nodes of [-1, 1] and the inverse of their Vandermonde matrix.
MfmaSincConst make_mfma_const()
{
    constexpr int n = kMfOrders;
    MfmaSincConst c{};
    double inv[n][2 * n];
    for (int i = 0; i < n; ++i) {
        c.node[i] = std::cos((2.0 * i + 1.0) * kPi / (2.0 * n));
        for (int j = 0; j < 2 * n; ++j)
            inv[i][j] = j < n ? std::pow(c.node[i], j) : (j - n == i ? 1.0 : 0.0);
    }
    // Gauss-Jordan on [V | I] with V[i][r] = z_i^r: a = V^-1 h gives p(z) = sum_r a_r z^r
    for (int p = 0; p < n; ++p) {
        int piv = p;
        for (int i = p + 1; i < n; ++i)
            if (std::fabs(inv[i][p]) > std::fabs(inv[piv][p]))
                piv = i;
        for (int j = 0; j < 2 * n; ++j)
            std::swap(inv[p][j], inv[piv][j]);
        const double d = inv[p][p];
        for (int j = 0; j < 2 * n; ++j)
            inv[p][j] /= d;
        for (int i = 0; i < n; ++i)
            if (i != p) {
                const double f = inv[i][p];
                for (int j = 0; j < 2 * n; ++j)
                    inv[i][j] -= f * inv[p][j];
            }
    }
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i)
            c.vinv[r * n + i] = inv[r][n + i];
    return c;
}

template <int H>
hipError_t build_table_h(const KaiserPoly &kp, void **dev, std::vector<void *> &allocs)
{
    const size_t bytes = (size_t)kPhaseRows * MfGeom<H>::bbytes;
    hipError_t e = hipMalloc(dev, bytes);
    if (e != hipSuccess)
        return e;
    allocs.push_back(*dev);
    const MfmaSincConst mc = make_mfma_const();
    unsigned char *t = static_cast<unsigned char *>(*dev);
    if (kp.n <= 24)
        hipLaunchKernelGGL((k_sinc_table<H, 24>), dim3(kPhaseRows), dim3(256), 0, 0, kp, mc, t);
    else if (kp.n <= 28)
        hipLaunchKernelGGL((k_sinc_table<H, 28>), dim3(kPhaseRows), dim3(256), 0, 0, kp, mc, t);
    else
        hipLaunchKernelGGL((k_sinc_table<H, 32>), dim3(kPhaseRows), dim3(256), 0, 0, kp, mc, t);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return hipStreamSynchronize(0);
}

// Per device: resident workgroups of k_sinc_mfma<H> per CU (the LDS limit raised once) and CUs.
struct MfDevice {
    bool ready = false;
    int per_cu = 0;
    int cus = 0;
};

template <int H>
hipError_t mf_device(MfDevice **out)
{
    static MfDevice devs[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    MfDevice &d = devs[dev];
    if (!d.ready) {
        const int lds = MfGeom<H>::bytes;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sinc_mfma<H>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.per_cu, k_sinc_mfma<H>, MfGeom<H>::threads, lds);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return e;
        if (d.per_cu < 1)
            d.per_cu = 1;
        d.ready = true;
    }
    *out = &d;
    return hipSuccess;
}

// Resident workgroups of the persistent grid: wg_per_cu per CU (0: as many as fit), at most
// what the kernel's resources allow.
template <int H>
hipError_t resident_wgs(int64_t *n, int wg_per_cu)
{
    MfDevice *d = nullptr;
    hipError_t e = mf_device<H>(&d);
    if (e == hipSuccess)
        *n = (int64_t)(wg_per_cu > 0 ? std::min(wg_per_cu, d->per_cu) : d->per_cu) * d->cus;
    return e;
}

// workspace: [ref: uint2 x n][list: uint2 x n][counts: u32 x 129 x chunks][phase: u8 x n]
int64_t sort_chunks(int64_t n) { return (n + kSortChunk - 1) / kSortChunk; }
size_t work_list_off(int64_t n) { return (size_t)n * 8; }
size_t work_counts_off(int64_t n) { return (size_t)n * 16; }
size_t work_phase_off(int64_t n) { return work_counts_off(n) + (size_t)sort_chunks(n) * kPhaseRows * 4; }

template <int H>
hipError_t launch_h(const SincJob *jobs_dev, const SincJob &inl, int njobs, int64_t max_out, int64_t ntiles,
                    void *work, const unsigned char *table, hipStream_t s, Profiler *prof, const TileStream *ts,
                    TileListMode mode, int wg_per_cu)
{
    MfDevice *d = nullptr;
    hipError_t e = mf_device<H>(&d);
    if (e != hipSuccess)
        return e;
    const size_t lds = MfGeom<H>::bytes;
    int64_t resident = 0;
    e = resident_wgs<H>(&resident, wg_per_cu);
    if (e != hipSuccess)
        return e;
    if (ntiles <= resident || !work) {
        if (mode == TileListMode::BuildOnly)
            return hipSuccess;  // no list on this path
        const int64_t nblk = (max_out + kMfOut - 1) / kMfOut;
        if (prof)
            prof->begin(kKSincMfma, s);
        hipLaunchKernelGGL(k_sinc_mfma<H>, dim3((unsigned)nblk, (unsigned)njobs), dim3(MfGeom<H>::threads), lds, s,
                           jobs_dev, inl, nullptr, (int64_t)0, table);
        e = hipGetLastError();
        if (prof)
            prof->end(s);
        return e;
    }
    // sorted tile list, then the persistent grid
    unsigned char *w = static_cast<unsigned char *>(work);
    uint2 *ref = reinterpret_cast<uint2 *>(w);
    uint2 *list = reinterpret_cast<uint2 *>(w + work_list_off(ntiles));
    unsigned char *phase = w + work_phase_off(ntiles);
    const int64_t tblk = (max_out + (int64_t)kMfOut * 256 - 1) / ((int64_t)kMfOut * 256);
    if (mode == TileListMode::RunOnly)
        goto run;
    {
    hipStream_t ls = s;
    if (ts) {
        ls = ts->stream;
        if (ts->after)
            e = hipStreamWaitEvent(ls, ts->after, 0);
        if (e != hipSuccess)
            return e;
    }
    if (prof)
        prof->begin(kKSincTiles, ls);
    hipLaunchKernelGGL(k_mf_tile_phase, dim3((unsigned)tblk, (unsigned)njobs), dim3(256), 0, ls, jobs_dev, ref, phase);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    unsigned *counts = reinterpret_cast<unsigned *>(w + work_counts_off(ntiles));
    const unsigned nch = (unsigned)sort_chunks(ntiles);
    hipLaunchKernelGGL(k_mf_tile_count, dim3(nch), dim3(256), 0, ls, phase, ntiles, counts);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mf_tile_scatter, dim3(nch), dim3(256), 0, ls, ref, phase, ntiles, counts, list);
        e = hipGetLastError();
    }
    if (prof)
        prof->end(ls);
    if (e == hipSuccess && ts) {
        e = hipEventRecord(ts->done, ls);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(s, ts->done, 0);
    }
    if (e != hipSuccess || mode == TileListMode::BuildOnly)
        return e;
    }
run:
    int64_t grid = resident;
    if (grid >= kXcds)
        grid -= grid % kXcds;
    if (prof)
        prof->begin(kKSincMfma, s);
    hipLaunchKernelGGL(k_sinc_mfma<H>, dim3((unsigned)grid), dim3(MfGeom<H>::threads), lds, s, jobs_dev, SincJob{},
                       list, ntiles, table);
    e = hipGetLastError();
    if (prof)
        prof->end(s);
    return e;
}

}  // namespace

bool sinc_mfma_eligible(double alpha, const rc_sinc &k)
{
    return k.window == RC_WIN_KAISER && (k.half_width == 64 || k.half_width == 128) &&
           std::fabs(alpha - 1.0) <= kSincMfmaMaxEps && make_kaiser_poly(k.kaiser_beta).n <= kMfKaiserTerms;
}

bool sinc_mfma_uses_list(int half_width, int64_t ntiles, int wg_per_cu)
{
    int64_t resident = 0;
    const hipError_t e =
        half_width == 64 ? resident_wgs<64>(&resident, wg_per_cu) : resident_wgs<128>(&resident, wg_per_cu);
    return e == hipSuccess && ntiles > resident;
}

size_t sinc_mfma_work_bytes(int64_t ntiles) { return work_phase_off(ntiles) + (size_t)ntiles; }

hipError_t build_sinc_mfma_table(int half_width, double beta, void **dev, std::vector<void *> &allocs)
{
    const KaiserPoly kp = make_kaiser_poly(beta);
    if (kp.n > kMfKaiserTerms)
        return hipErrorInvalidValue;
    if (half_width == 64)
        return build_table_h<64>(kp, dev, allocs);
    if (half_width == 128)
        return build_table_h<128>(kp, dev, allocs);
    return hipErrorInvalidValue;
}

hipError_t launch_sinc_mfma(const SincJob *jobs_dev, const SincJob *job_inline, int njobs, int64_t max_out,
                            int64_t ntiles, void *work, int half_width, const void *table, hipStream_t s,
                            Profiler *prof, const TileStream *ts, TileListMode mode, int wg_per_cu)
{
    if (njobs <= 0 || max_out <= 0)
        return hipSuccess;
    const int64_t nblk = (max_out + kMfOut - 1) / kMfOut;
    // the list holds 32-bit job and tile indices and is sorted in 32-bit counters
    if (nblk > 0x7fffffff || njobs > 65535 || !table || ntiles <= 0 || ntiles > 0x7fffffff)
        return hipErrorInvalidValue;
    if (work && !jobs_dev)
        return hipErrorInvalidValue;  // the list kernels read the job array
    const SincJob inl = job_inline ? *job_inline : SincJob{};
    const unsigned char *t = static_cast<const unsigned char *>(table);
    return half_width == 64
               ? launch_h<64>(jobs_dev, inl, njobs, max_out, ntiles, work, t, s, prof, ts, mode, wg_per_cu)
               : launch_h<128>(jobs_dev, inl, njobs, max_out, ntiles, work, t, s, prof, ts, mode, wg_per_cu);
}

}  // namespace rc
