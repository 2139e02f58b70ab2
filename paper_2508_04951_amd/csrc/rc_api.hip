// rc_api.hip -- the extern "C" entry points of librc.so declared in include/rc.h:
// argument validation, the per-device context, and dispatch to the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rc_internal.h"

namespace {

using rc::FftPlan;
using rc::IonoJob;
using rc::SincJob;

rc_status fail(rc_context ctx, rc_status st, const std::string &why)
{
    if (ctx)
        ctx->last_error = why;
    return st;
}

rc_status device_fail(rc_context ctx, hipError_t e, const char *where)
{
    return fail(ctx, RC_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool overlaps(const void *a, int64_t abytes, const void *b, int64_t bbytes)
{
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// Power-of-two lengths run the multi-level FFT directly (up to 2^24); other lengths run
// Bluestein at the power of two m >= 2n - 1 (so up to 2^23).
constexpr int64_t kMaxIonoLength = int64_t(1) << 24;
int64_t iono_plan_length(int64_t n)
{
    if (is_pow2(n))
        return n;
    int64_t m = 1;
    while (m < 2 * n - 1)
        m <<= 1;
    return m;
}

rc_status check_sinc(rc_context ctx, const rc_sinc *k)
{
    if (!k)
        return fail(ctx, RC_ERR_INVALID_ARG, "sinc kernel descriptor is NULL");
    if (k->half_width < 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "half_width must be >= 0");
    if (k->window != RC_WIN_KAISER && k->window != RC_WIN_RECT && k->window != RC_WIN_PAPER)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown window");
    if (k->window == RC_WIN_KAISER && !(k->kaiser_beta >= 0.0 && k->kaiser_beta <= 40.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "kaiser_beta must be in [0, 40]");
    return RC_OK;
}

// Current device of the calling thread set to the context's device for the call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

// Stage `bytes` of descriptors to the device on `s`, in the next slot of the context's ring, with
// `extra` more bytes of device workspace after them (from offset align256(bytes)).  A slot is
// reused only after the work that read it has completed, so the host may run up to
// kDescSlots - 1 calls ahead of the device.
rc_status stage_descriptors(rc_context ctx, const void *host, size_t bytes, size_t extra, hipStream_t s,
                            const void **dev_out)
{
    auto &slot = ctx->desc[ctx->desc_next];
    hipError_t e;
    if (slot.pending) {
        e = hipEventSynchronize(slot.done);
        if (e != hipSuccess)
            return device_fail(ctx, e, "waiting for an earlier call");
        slot.pending = false;
    }
    const size_t dev_bytes = extra ? ((bytes + 255) & ~(size_t)255) + extra : bytes;
    auto grow = [](size_t need) {
        size_t cap = 1 << 16;
        while (cap < need)
            cap <<= 1;
        return cap;
    };
    if (bytes > slot.host_cap) {
        if (slot.host)
            (void)hipHostFree(slot.host);
        slot.host = nullptr;
        slot.host_cap = 0;
        const size_t cap = grow(bytes);
        if (hipHostMalloc(&slot.host, cap, hipHostMallocDefault) != hipSuccess)
            return fail(ctx, RC_ERR_OUT_OF_MEMORY, "descriptor staging allocation failed");
        slot.host_cap = cap;
    }
    if (dev_bytes > slot.dev_cap) {
        if (slot.dev)
            (void)hipFree(slot.dev);
        slot.dev = nullptr;
        slot.dev_cap = 0;
        const size_t cap = grow(dev_bytes);
        if (hipMalloc(&slot.dev, cap) != hipSuccess)
            return fail(ctx, RC_ERR_OUT_OF_MEMORY, "descriptor workspace allocation failed");
        slot.dev_cap = cap;
    }
    if (bytes) {
        std::memcpy(slot.host, host, bytes);
        e = hipMemcpyAsync(slot.dev, slot.host, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return device_fail(ctx, e, "descriptor upload");
    }
    *dev_out = slot.dev;
    return RC_OK;
}

// The work that reads the slot filled by the last stage_descriptors() is now enqueued on `s`.
rc_status mark_descriptors_used(rc_context ctx, hipStream_t s)
{
    auto &slot = ctx->desc[ctx->desc_next];
    hipError_t e = hipEventRecord(slot.done, s);
    if (e != hipSuccess)
        return device_fail(ctx, e, "descriptor event");
    slot.pending = true;
    ctx->desc_next = (ctx->desc_next + 1) % rc_context_s::kDescSlots;
    return RC_OK;
}

rc_status get_plan(rc_context ctx, int64_t n, const FftPlan **out)
{
    auto it = ctx->plans.find(n);
    if (it == ctx->plans.end()) {
        FftPlan plan;
        hipError_t e = rc::build_fft_plan(n, plan, ctx->allocs);
        if (e == hipErrorInvalidValue)
            return fail(ctx, RC_ERR_UNSUPPORTED, "transform length " + std::to_string(n) + " not supported");
        if (e != hipSuccess)
            return device_fail(ctx, e, "building FFT tables");
        it = ctx->plans.emplace(n, plan).first;
    }
    *out = &it->second;
    return RC_OK;
}

rc_status get_mfma_table(rc_context ctx, const rc_sinc &k, const void **out)
{
    const auto key = std::make_pair((int)k.half_width, k.kaiser_beta);
    auto it = ctx->mfma_tables.find(key);
    if (it == ctx->mfma_tables.end()) {
        void *t = nullptr;
        hipError_t e = rc::build_sinc_mfma_table(k.half_width, k.kaiser_beta, &t, ctx->allocs);
        if (e != hipSuccess)
            return device_fail(ctx, e, "building the matrix-core weight table");
        it = ctx->mfma_tables.emplace(key, t).first;
    }
    *out = it->second;
    return RC_OK;
}

double phase_numerator(double tec, int32_t direction)
{
    const double k2 = rc_k2_per_tec() * tec;
    const double s = (direction == RC_DISTORT) ? 1.0 : -1.0;
    return s * 4.0 * rc::kPi * k2 / rc::kC;
}

rc::Profiler *prof_of(rc_context ctx) { return ctx->prof.on ? &ctx->prof : nullptr; }

enum class SincPath { Mfma, Fast, Direct };

SincPath sinc_path(rc_context ctx, double alpha, const rc_sinc &k)
{
    if (ctx->sinc_engine == RC_SINC_DIRECT)
        return SincPath::Direct;
    if (ctx->sinc_engine == RC_SINC_AUTO && rc::sinc_mfma_eligible(alpha, k))
        return SincPath::Mfma;
    if (rc::sinc_fast_eligible(alpha, k))
        return SincPath::Fast;
    return SincPath::Direct;
}

int64_t taps_per_output(const rc_sinc &k, int64_t n_in)
{
    if (k.half_width == 0)
        return n_in;
    return k.window == RC_WIN_PAPER ? 2 * (int64_t)k.half_width + 1 : 2 * (int64_t)k.half_width;
}

}  // namespace

extern "C" {

const char *rc_status_string(rc_status status)
{
    switch (status) {
    case RC_OK: return "RC_OK";
    case RC_ERR_INVALID_ARG: return "RC_ERR_INVALID_ARG";
    case RC_ERR_UNSUPPORTED: return "RC_ERR_UNSUPPORTED";
    case RC_ERR_OUT_OF_MEMORY: return "RC_ERR_OUT_OF_MEMORY";
    case RC_ERR_DEVICE: return "RC_ERR_DEVICE";
    case RC_ERR_BUSY: return "RC_ERR_BUSY";
    }
    return "RC_ERR_UNKNOWN";
}

double rc_alpha_from_vr(double v_r_mps)
{
    if (!(std::fabs(v_r_mps) < rc::kC))
        return NAN;
    // (1 + v/c)/(1 - v/c).  For |v| < c/4 it is evaluated as 1 + 2v/(c - v), which keeps
    // alpha - 1 at full relative precision; closer to c the plain quotient avoids the
    // cancellation of 1 + 2v/(c - v).
    if (std::fabs(v_r_mps) < 0.25 * rc::kC)
        return 1.0 + 2.0 * v_r_mps / (rc::kC - v_r_mps);
    return (rc::kC + v_r_mps) / (rc::kC - v_r_mps);
}

double rc_k2_per_tec(void)
{
    return rc::kECharge * rc::kECharge / (8.0 * rc::kPi * rc::kPi * rc::kMe * rc::kEps0);
}

rc_status rc_create(int hip_device, rc_context *out)
{
    if (!out)
        return RC_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return RC_ERR_INVALID_ARG;
    rc_context ctx = new (std::nothrow) rc_context_s();
    if (!ctx)
        return RC_ERR_OUT_OF_MEMORY;
    ctx->device = hip_device;
    DeviceGuard g(hip_device);
    hipError_t e = rc::make_base_twiddles(&ctx->tw4096);
    for (auto &slot : ctx->desc)
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (auto &slot : ctx->desc)
            if (slot.done)
                (void)hipEventDestroy(slot.done);
        if (ctx->tw4096)
            (void)hipFree(ctx->tw4096);
        delete ctx;
        return RC_ERR_DEVICE;
    }
    *out = ctx;
    return RC_OK;
}

rc_status rc_destroy(rc_context ctx)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    rc_status st = RC_OK;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        DeviceGuard g(ctx->device);
        if (hipDeviceSynchronize() != hipSuccess)
            st = RC_ERR_DEVICE;
        for (void *p : ctx->allocs)
            (void)hipFree(p);
        if (ctx->tw4096)
            (void)hipFree(ctx->tw4096);
        for (auto &slot : ctx->desc) {
            if (slot.dev)
                (void)hipFree(slot.dev);
            if (slot.host)
                (void)hipHostFree(slot.host);
            if (slot.done)
                (void)hipEventDestroy(slot.done);
        }
        ctx->prof.release();
    }
    delete ctx;
    return st;
}

const char *rc_last_error(rc_context ctx)
{
    return ctx ? ctx->last_error.c_str() : "NULL context";
}

rc_status rc_sync(rc_context ctx, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return device_fail(ctx, e, "rc_sync");
    return RC_OK;
}

rc_status correct_doppler(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y, int64_t n_out,
                          double fs_hz, double alpha, const rc_sinc *k, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_sinc(ctx, k);
    if (st != RC_OK)
        return st;
    if (!x || !y)
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL sample pointer");
    if (n_in <= 0 || n_out <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "n_in and n_out must be > 0");
    if (!(std::isfinite(fs_hz) && fs_hz > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "fs_hz must be finite and > 0");
    if (!(std::isfinite(alpha) && alpha > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "alpha must be finite and > 0");
    if (overlaps(x, n_in * 8, y, n_out * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SincJob job{reinterpret_cast<const float2 *>(x), reinterpret_cast<float2 *>(y), n_in, n_out, alpha, 0};
    const rc::KaiserPoly kp = rc::make_kaiser_poly(k->window == RC_WIN_KAISER ? k->kaiser_beta : 0.0);
    hipError_t e;
    switch (sinc_path(ctx, alpha, *k)) {
    case SincPath::Mfma: {
        const void *table = nullptr;
        rc_status ts = get_mfma_table(ctx, *k, &table);
        if (ts != RC_OK)
            return ts;
        const int64_t ntiles = (n_out + rc::kSincMfmaTile - 1) / rc::kSincMfmaTile;
        if (!rc::sinc_mfma_uses_list(k->half_width, ntiles)) {
            e = rc::launch_sinc_mfma(nullptr, &job, 1, n_out, ntiles, nullptr, k->half_width, table, s,
                                     prof_of(ctx));
            break;
        }
        // a long pulse: the job descriptor and the tile list go to a staging slot
        const void *dev = nullptr;
        ts = stage_descriptors(ctx, &job, sizeof job, rc::sinc_mfma_work_bytes(ntiles), s, &dev);
        if (ts != RC_OK)
            return ts;
        char *devc = static_cast<char *>(const_cast<void *>(dev));
        e = rc::launch_sinc_mfma(reinterpret_cast<const SincJob *>(devc), nullptr, 1, n_out, ntiles, devc + 256,
                                 k->half_width, table, s, prof_of(ctx));
        ts = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && ts != RC_OK)
            return ts;
        break;
    }
    case SincPath::Fast:
        e = rc::launch_sinc_fast(nullptr, &job, 1, n_out, k->half_width, kp, s, prof_of(ctx));
        break;
    default:
        e = rc::launch_sinc_direct(nullptr, &job, 1, n_out, *k, kp, taps_per_output(*k, n_in), s, prof_of(ctx));
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_doppler launch");
    return RC_OK;
}

rc_status correct_ionosphere(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n, double fs_hz,
                             double carrier_hz, double tec_el_per_m2, int32_t direction, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (!x || !y)
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL sample pointer");
    if (n <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "n must be > 0");
    if (!(std::isfinite(fs_hz) && fs_hz > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "fs_hz must be finite and > 0");
    if (!std::isfinite(carrier_hz))
        return fail(ctx, RC_ERR_INVALID_ARG, "carrier_hz must be finite");
    if (!(std::isfinite(tec_el_per_m2) && tec_el_per_m2 >= 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "tec must be finite and >= 0");
    if (direction != RC_CORRECT && direction != RC_DISTORT)
        return fail(ctx, RC_ERR_INVALID_ARG, "direction must be RC_CORRECT or RC_DISTORT");
    if (x != y && overlaps(x, n * 8, y, n * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y partially overlap");
    if (n > kMaxIonoLength)
        return fail(ctx, RC_ERR_UNSUPPORTED, "n above 2^24 (power of two) or 2^23 (other lengths)");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double phase = phase_numerator(tec_el_per_m2, direction);
    const float2 *xf = reinterpret_cast<const float2 *>(x);
    float2 *yf = reinterpret_cast<float2 *>(y);
    const FftPlan *plan = nullptr;
    rc_status st = get_plan(ctx, iono_plan_length(n), &plan);
    if (st != RC_OK)
        return st;
    hipError_t e;
    if (is_pow2(n)) {
        const IonoJob job{xf, yf, phase, carrier_hz, fs_hz, nullptr};
        e = rc::launch_iono(*plan, ctx->tw4096, nullptr, &job, 1, s, prof_of(ctx));
    } else {
        // Bluestein: its workspace is a staging slot, reused only after this work completes
        const void *dev = nullptr;
        st = stage_descriptors(ctx, nullptr, 0, rc::bluestein_work_bytes(n), s, &dev);
        if (st != RC_OK)
            return st;
        e = rc::launch_iono_bluestein(n, *plan, ctx->tw4096, xf, yf, phase, carrier_hz, fs_hz,
                                      const_cast<void *>(dev), s, prof_of(ctx));
        st = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && st != RC_OK)
            return st;
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_ionosphere launch");
    return RC_OK;
}

namespace {

// correct_pulse_batch with the context lock held (also the per-hypothesis Doppler bank)
rc_status pulse_batch_locked(rc_context ctx, const rc_c64 *x_packed, int64_t x_len, rc_c64 *y_packed,
                             int64_t y_len, const rc_pulse *pulses, int32_t count, const rc_sinc *k, void *stream)
{
    rc_status st = check_sinc(ctx, k);
    if (st != RC_OK)
        return st;
    if (count < 0 || (count > 0 && (!pulses || !x_packed || !y_packed)))
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL pointer or negative count");
    if (count == 0)
        return RC_OK;
    if (x_len <= 0 || y_len <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "buffer lengths must be > 0");
    if (overlaps(x_packed, x_len * 8, y_packed, y_len * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "input and output buffers overlap");
    // validate every pulse; output ranges must be pairwise disjoint
    std::vector<std::pair<int64_t, int64_t>> outs;
    outs.reserve((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const rc_pulse &p = pulses[i];
        const std::string at = "pulse " + std::to_string(i) + ": ";
        if (p.n_in <= 0 || p.n_out <= 0 || p.off_in < 0 || p.off_out < 0 || p.off_in > x_len - p.n_in ||
            p.off_out > y_len - p.n_out)
            return fail(ctx, RC_ERR_INVALID_ARG, at + "range outside its buffer");
        if ((p.flags & ~(uint32_t)(RC_DO_DOPPLER | RC_DO_IONO)) != 0)
            return fail(ctx, RC_ERR_INVALID_ARG, at + "unknown flag bits");
        if (!(std::isfinite(p.fs_hz) && p.fs_hz > 0.0))
            return fail(ctx, RC_ERR_INVALID_ARG, at + "fs_hz must be finite and > 0");
        if ((p.flags & RC_DO_DOPPLER) && !(std::isfinite(p.alpha) && p.alpha > 0.0))
            return fail(ctx, RC_ERR_INVALID_ARG, at + "alpha must be finite and > 0");
        if (!(p.flags & RC_DO_DOPPLER) && p.n_out != p.n_in)
            return fail(ctx, RC_ERR_INVALID_ARG, at + "n_out must equal n_in without RC_DO_DOPPLER");
        if (p.flags & RC_DO_IONO) {
            if (!(std::isfinite(p.tec_el_per_m2) && p.tec_el_per_m2 >= 0.0) || !std::isfinite(p.carrier_hz))
                return fail(ctx, RC_ERR_INVALID_ARG, at + "tec must be finite and >= 0, carrier finite");
            if (p.direction != RC_CORRECT && p.direction != RC_DISTORT)
                return fail(ctx, RC_ERR_INVALID_ARG, at + "bad direction");
            if (p.n_out > kMaxIonoLength || (!is_pow2(p.n_out) && 2 * p.n_out - 1 > kMaxIonoLength))
                return fail(ctx, RC_ERR_UNSUPPORTED, at + "iono length above 2^24 (power of two) or 2^23 (other)");
        }
        outs.emplace_back(p.off_out, p.off_out + p.n_out);
    }
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].first < outs[i - 1].second)
            return fail(ctx, RC_ERR_INVALID_ARG, "output ranges overlap");

    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float2 *xb = reinterpret_cast<const float2 *>(x_packed);
    float2 *yb = reinterpret_cast<float2 *>(y_packed);

    // Group the work: fast-path Doppler jobs, generic Doppler jobs, plain copies, and the
    // ionospheric jobs by transform length (one launch sequence per length).
    std::vector<SincJob> mfma, fast, direct;
    int64_t mfma_max = 0, fast_max = 0, direct_max = 0, direct_taps = 0;
    std::map<int64_t, std::vector<IonoJob>> iono;
    std::vector<int32_t> copies;
    for (int32_t i = 0; i < count; ++i) {
        const rc_pulse &p = pulses[i];
        if (p.flags & RC_DO_DOPPLER) {
            const SincJob j{xb + p.off_in, yb + p.off_out, p.n_in, p.n_out, p.alpha, 0};
            const SincPath path = sinc_path(ctx, p.alpha, *k);
            if (path == SincPath::Mfma) {
                mfma.push_back(j);
                mfma_max = std::max(mfma_max, p.n_out);
            } else if (path == SincPath::Fast) {
                fast.push_back(j);
                fast_max = std::max(fast_max, p.n_out);
            } else {
                direct.push_back(j);
                direct_max = std::max(direct_max, p.n_out);
                direct_taps = std::max(direct_taps, taps_per_output(*k, p.n_in));
            }
        } else if (!(p.flags & RC_DO_IONO)) {
            copies.push_back(i);
        }
        if (p.flags & RC_DO_IONO) {
            const float2 *src = (p.flags & RC_DO_DOPPLER) ? yb + p.off_out : xb + p.off_in;
            iono[p.n_out].push_back(IonoJob{src, yb + p.off_out, phase_numerator(p.tec_el_per_m2, p.direction),
                                            p.carrier_hz, p.fs_hz});
        }
    }
    if (mfma.size() > 65535 || fast.size() > 65535 || direct.size() > 65535)
        return fail(ctx, RC_ERR_UNSUPPORTED, "more than 65535 pulses of one kind in a batch");
    size_t bs_work = 0;  // Bluestein workspace: one region, reused by the pulses in stream order
    for (auto &kv : iono) {
        const FftPlan *plan = nullptr;
        st = get_plan(ctx, iono_plan_length(kv.first), &plan);
        if (st != RC_OK)
            return st;
        if (!is_pow2(kv.first))
            bs_work = std::max(bs_work, rc::bluestein_work_bytes(kv.first));
    }
    const void *mfma_table = nullptr;
    int64_t mfma_tiles = 0;
    size_t mfma_work = 0;
    if (!mfma.empty()) {
        st = get_mfma_table(ctx, *k, &mfma_table);
        if (st != RC_OK)
            return st;
        for (SincJob &j : mfma) {
            j.tile0 = mfma_tiles;
            mfma_tiles += (j.n_out + rc::kSincMfmaTile - 1) / rc::kSincMfmaTile;
        }
        if (mfma_tiles > 0x7fffffff)
            return fail(ctx, RC_ERR_UNSUPPORTED, "more than 2^31 - 1 matrix-core tiles in a batch");
        if (rc::sinc_mfma_uses_list(k->half_width, mfma_tiles))
            mfma_work = rc::sinc_mfma_work_bytes(mfma_tiles);
    }

    // one descriptor upload: [mfma | fast | direct | iono groups...], then the tile-list workspace
    std::vector<char> blob;
    auto append = [&](const void *p, size_t bytes) {
        const size_t off = (blob.size() + 15) & ~(size_t)15;
        blob.resize(off + bytes);
        std::memcpy(blob.data() + off, p, bytes);
        return off;
    };
    const size_t off_mfma = mfma.empty() ? 0 : append(mfma.data(), mfma.size() * sizeof(SincJob));
    const size_t off_fast = fast.empty() ? 0 : append(fast.data(), fast.size() * sizeof(SincJob));
    const size_t off_direct = direct.empty() ? 0 : append(direct.data(), direct.size() * sizeof(SincJob));
    std::vector<size_t> off_iono;
    for (auto &kv : iono)  // Bluestein lengths run from the host copies of their descriptors
        off_iono.push_back(is_pow2(kv.first) ? append(kv.second.data(), kv.second.size() * sizeof(IonoJob)) : 0);
    // device workspace after the descriptors: [tile list][Bluestein]
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t extra = mfma_work || bs_work ? al(mfma_work) + bs_work : 0;
    const void *dev = nullptr;
    if (!blob.empty() || extra) {
        st = stage_descriptors(ctx, blob.data(), blob.size(), extra, s, &dev);
        if (st != RC_OK)
            return st;
    }
    char *devc = static_cast<char *>(const_cast<void *>(dev));
    char *wbase = extra ? devc + al(blob.size()) : nullptr;
    void *work = mfma_work ? wbase : nullptr;
    void *bwork = bs_work ? wbase + al(mfma_work) : nullptr;
    // from here on the slot is in use: mark it whatever happens
    struct SlotMark {
        rc_context ctx;
        hipStream_t s;
        bool armed;
        ~SlotMark()
        {
            if (armed)
                (void)mark_descriptors_used(ctx, s);
        }
    } slot_mark{ctx, s, dev != nullptr};
    hipError_t e = hipSuccess;
    for (int32_t i : copies) {
        const rc_pulse &p = pulses[i];
        e = hipMemcpyAsync(yb + p.off_out, xb + p.off_in, (size_t)p.n_in * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return device_fail(ctx, e, "copy");
    }
    const rc::KaiserPoly kp = rc::make_kaiser_poly(k->window == RC_WIN_KAISER ? k->kaiser_beta : 0.0);
    if (!mfma.empty())
        e = rc::launch_sinc_mfma(reinterpret_cast<const SincJob *>(devc + off_mfma), nullptr, (int)mfma.size(),
                                 mfma_max, mfma_tiles, work, k->half_width, mfma_table, s, prof_of(ctx));
    if (e == hipSuccess && !fast.empty())
        e = rc::launch_sinc_fast(reinterpret_cast<const SincJob *>(devc + off_fast), nullptr, (int)fast.size(),
                                 fast_max, k->half_width, kp, s, prof_of(ctx));
    if (e == hipSuccess && !direct.empty())
        e = rc::launch_sinc_direct(reinterpret_cast<const SincJob *>(devc + off_direct), nullptr,
                                   (int)direct.size(), direct_max, *k, kp, direct_taps, s, prof_of(ctx));
    if (e != hipSuccess)
        return device_fail(ctx, e, "batch Doppler launch");
    size_t gi = 0;
    for (auto &kv : iono) {
        const FftPlan *plan = nullptr;
        st = get_plan(ctx, iono_plan_length(kv.first), &plan);
        if (st != RC_OK)
            return st;
        if (!is_pow2(kv.first)) {
            ++gi;
            for (const IonoJob &jb : kv.second) {
                e = rc::launch_iono_bluestein(kv.first, *plan, ctx->tw4096, jb.x, jb.y, jb.phase_num, jb.carrier,
                                              jb.fs, bwork, s, prof_of(ctx));
                if (e != hipSuccess)
                    return device_fail(ctx, e, "batch ionosphere launch");
            }
            continue;
        }
        const IonoJob *jd = reinterpret_cast<const IonoJob *>(devc + off_iono[gi++]);
        // at most 65535 pulses per launch keeps every grid dimension in range
        for (size_t b = 0; b < kv.second.size(); b += 65535) {
            const int nj = (int)std::min<size_t>(65535, kv.second.size() - b);
            e = rc::launch_iono(*plan, ctx->tw4096, jd + b, nullptr, nj, s, prof_of(ctx));
            if (e != hipSuccess)
                return device_fail(ctx, e, "batch ionosphere launch");
        }
    }
    if (dev) {
        slot_mark.armed = false;
        return mark_descriptors_used(ctx, s);
    }
    return RC_OK;
}

rc_status get_farrow_coef(rc_context ctx, const rc_sinc &k, const float **out)
{
    const double beta = k.window == RC_WIN_KAISER ? k.kaiser_beta : 0.0;
    const auto key = std::make_pair(std::make_pair((int)k.half_width, (int)k.window), beta);
    auto it = ctx->farrow_coefs.find(key);
    if (it == ctx->farrow_coefs.end()) {
        void *t = nullptr;
        hipError_t e = rc::build_farrow_coef(k, &t, ctx->allocs);
        if (e != hipSuccess)
            return device_fail(ctx, e, "building the filter-bank coefficients");
        it = ctx->farrow_coefs.emplace(key, t).first;
    }
    *out = static_cast<const float *>(it->second);
    return RC_OK;
}

}  // namespace

rc_status correct_pulse_batch(rc_context ctx, const rc_c64 *x_packed, int64_t x_len, rc_c64 *y_packed,
                              int64_t y_len, const rc_pulse *pulses, int32_t count, const rc_sinc *k,
                              void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    return pulse_batch_locked(ctx, x_packed, x_len, y_packed, y_len, pulses, count, k, stream);
}

rc_status correct_doppler_bank(rc_context ctx, const rc_c64 *x, int64_t n, rc_c64 *y, int64_t n_out, double fs_hz,
                               const double *alphas, int32_t n_hyp, const rc_sinc *k, int32_t mode, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_sinc(ctx, k);
    if (st != RC_OK)
        return st;
    if (!x || !y || !alphas)
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL pointer");
    if (n <= 0 || n_out <= 0 || n_hyp <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "n, n_out and n_hyp must be > 0");
    if (!(std::isfinite(fs_hz) && fs_hz > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "fs_hz must be finite and > 0");
    if (mode != RC_BANK_AUTO && mode != RC_BANK_FARROW && mode != RC_BANK_PER_HYPOTHESIS)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown bank mode");
    for (int32_t h = 0; h < n_hyp; ++h)
        if (!(std::isfinite(alphas[h]) && alphas[h] > 0.0))
            return fail(ctx, RC_ERR_INVALID_ARG, "hypothesis " + std::to_string(h) + ": alpha must be finite and > 0");
    if (n_out > INT64_MAX / 8 / n_hyp)
        return fail(ctx, RC_ERR_INVALID_ARG, "output size overflows");
    if (overlaps(x, n * 8, y, n_out * n_hyp * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    const bool farrow = mode != RC_BANK_PER_HYPOTHESIS && rc::farrow_eligible(*k, alphas, n_hyp);
    if (mode == RC_BANK_FARROW && !farrow)
        return fail(ctx, RC_ERR_UNSUPPORTED,
                    "the filter bank needs a Kaiser or rectangular window, 1 <= H <= 256 and 0 < alpha <= 2");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!farrow) {
        std::vector<rc_pulse> pulses((size_t)n_hyp);
        for (int32_t h = 0; h < n_hyp; ++h) {
            rc_pulse &p = pulses[(size_t)h];
            p = rc_pulse{};
            p.off_in = 0;
            p.n_in = n;
            p.off_out = (int64_t)h * n_out;
            p.n_out = n_out;
            p.fs_hz = fs_hz;
            p.alpha = alphas[h];
            p.carrier_hz = 0.0;
            p.flags = RC_DO_DOPPLER;
            p.direction = RC_CORRECT;
        }
        return pulse_batch_locked(ctx, x, n, y, n_out * n_hyp, pulses.data(), n_hyp, k, stream);
    }
    const float *coef = nullptr;
    st = get_farrow_coef(ctx, *k, &coef);
    if (st != RC_OK)
        return st;
    const rc::FarrowPlan plan = rc::plan_farrow_bank(n, n_out, k->half_width, alphas, n_hyp);
    if (plan.lds_bytes > 160 * 1024)
        return fail(ctx, RC_ERR_UNSUPPORTED, "filter-bank tile exceeds LDS");
    std::vector<char> desc(rc::farrow_desc_bytes(plan));
    rc::farrow_pack_desc(plan, desc.data());
    const void *dev = nullptr;
    st = stage_descriptors(ctx, desc.data(), desc.size(), plan.z_bytes, s, &dev);
    if (st != RC_OK)
        return st;
    char *devc = static_cast<char *>(const_cast<void *>(dev));
    hipError_t e = rc::launch_farrow_bank(plan, reinterpret_cast<const float2 *>(x), n, reinterpret_cast<float2 *>(y),
                                          n_out, k->half_width, coef, devc, devc + ((desc.size() + 255) & ~(size_t)255),
                                          s, prof_of(ctx));
    st = mark_descriptors_used(ctx, s);
    if (e != hipSuccess)
        return device_fail(ctx, e, "Doppler bank launch");
    return st;
}

rc_status rc_set_sinc_engine(rc_context ctx, int32_t engine)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    if (engine != RC_SINC_AUTO && engine != RC_SINC_VALU && engine != RC_SINC_DIRECT)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown sinc engine");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->sinc_engine = engine;
    return RC_OK;
}

rc_status rc_profile_enable(rc_context ctx, int enable)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prof.on = enable != 0;
    return RC_OK;
}

rc_status rc_profile_read(rc_context ctx, const char *kernel, double *total_ms, int64_t *launches)
{
    if (!ctx || !kernel || !total_ms || !launches)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    int grp = -1;
    for (int i = 0; i < rc::kKGroups; ++i)
        if (std::strcmp(kernel, rc::kKernelNames[i]) == 0)
            grp = i;
    if (grp < 0)
        return fail(ctx, RC_ERR_INVALID_ARG, std::string("unknown kernel name ") + kernel);
    hipError_t e = ctx->prof.collect();
    if (e != hipSuccess)
        return device_fail(ctx, e, "rc_profile_read");
    *total_ms = ctx->prof.total_ms[grp];
    *launches = ctx->prof.launches[grp];
    ctx->prof.total_ms[grp] = 0.0;
    ctx->prof.launches[grp] = 0;
    return RC_OK;
}

}  // extern "C"

namespace rc {

const char *const kKernelNames[kKGroups] = {"k_sinc_fast", "k_sinc_direct", "k_fft_strided_fwd",
                                            "k_fft_rows_iono", "k_fft_strided_inv", "k_sinc_mfma",
                                            "k_mf_tile_list", "k_bluestein", "k_farrow_z", "k_farrow_bank"};

hipEvent_t Profiler::take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

void Profiler::begin(int group, hipStream_t s)
{
    open_group = group;
    open_a = take();
    if (open_a)
        (void)hipEventRecord(open_a, s);
}

void Profiler::end(hipStream_t s)
{
    hipEvent_t b = take();
    if (open_a && b && hipEventRecord(b, s) == hipSuccess) {
        spans.push_back(Span{open_group, open_a, b});
    } else {
        if (open_a)
            pool.push_back(open_a);
        if (b)
            pool.push_back(b);
    }
    open_a = nullptr;
    open_group = -1;
}

hipError_t Profiler::collect()
{
    hipError_t first = hipSuccess;
    for (const Span &sp : spans) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(sp.b);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, sp.a, sp.b);
        if (e == hipSuccess) {
            total_ms[sp.group] += ms;
            launches[sp.group] += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        pool.push_back(sp.a);
        pool.push_back(sp.b);
    }
    spans.clear();
    return first;
}

void Profiler::release()
{
    (void)collect();
    for (hipEvent_t e : pool)
        (void)hipEventDestroy(e);
    pool.clear();
}

}  // namespace rc
