// rc_api.hip -- the extern "C" entry points of librc.so declared in include/rc.h:
// argument validation, the per-device context, and dispatch to the HIP kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rc_internal.h"

namespace {

using rc::FftPlan;
using rc::IonoJob;
using rc::PhaseNum;
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
// Waits until the next ring slot is free and sizes it for `bytes` of descriptors plus `extra`
// bytes of device workspace (at the next 256-byte boundary); returns the slot's pinned host
// buffer and its device buffer.
rc_status reserve_descriptors(rc_context ctx, size_t bytes, size_t extra, void **host_out, char **dev_out)
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
        size_t cap = grow(dev_bytes);
        if (ctx->mem_budget > 0) {
            // Under a budget every slot holds exactly what its last call needed, and the slots
            // whose work has completed give their workspace back when the total would exceed the
            // budget; the slots still in use keep theirs.  This one is replaced.
            cap = dev_bytes;
            const size_t budget = (size_t)ctx->mem_budget;
            auto others = [&] {
                size_t o = 0;
                for (int i = 0; i < rc_context_s::kDescSlots; ++i)
                    if (i != ctx->desc_next)
                        o += ctx->desc[i].dev_cap;
                return o;
            };
            if (others() + cap > budget) {
                for (int i = 0; i < rc_context_s::kDescSlots; ++i) {
                    auto &o = ctx->desc[i];
                    if (i == ctx->desc_next || !o.dev)
                        continue;
                    if (o.pending && hipEventQuery(o.done) != hipSuccess)
                        continue;  // still in use (or failed: kept until its event is waited for)
                    (void)hipFree(o.dev);
                    o.dev = nullptr;
                    o.dev_cap = 0;
                    o.pending = false;
                }
            }
            if (others() + cap > budget)
                return fail(ctx, RC_ERR_OUT_OF_MEMORY,
                            "workspace of " + std::to_string(others() + cap) +
                                " bytes would exceed the memory budget of " + std::to_string(budget) +
                                " (rc_set_mem_budget)");
        }
        if (slot.dev)
            (void)hipFree(slot.dev);
        slot.dev = nullptr;
        slot.dev_cap = 0;
        if (hipMalloc(&slot.dev, cap) != hipSuccess)
            return fail(ctx, RC_ERR_OUT_OF_MEMORY, "descriptor workspace allocation failed");
        slot.dev_cap = cap;
    }
    *host_out = slot.host;
    *dev_out = static_cast<char *>(slot.dev);
    return RC_OK;
}

// Uploads the first `bytes` of the reserved slot's host buffer on the copy stream; `s` waits for it.
rc_status upload_descriptors(rc_context ctx, size_t bytes, hipStream_t s)
{
    if (!bytes)
        return RC_OK;
    auto &slot = ctx->desc[ctx->desc_next];
    hipError_t e = hipMemcpyAsync(slot.dev, slot.host, bytes, hipMemcpyHostToDevice, ctx->copy_stream);
    if (e == hipSuccess)
        e = hipEventRecord(slot.uploaded, ctx->copy_stream);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(s, slot.uploaded, 0);
    if (e != hipSuccess)
        return device_fail(ctx, e, "descriptor upload");
    return RC_OK;
}

rc_status stage_descriptors(rc_context ctx, const void *host, size_t bytes, size_t extra, hipStream_t s,
                            const void **dev_out)
{
    void *h = nullptr;
    char *d = nullptr;
    rc_status st = reserve_descriptors(ctx, bytes, extra, &h, &d);
    if (st != RC_OK)
        return st;
    if (bytes)
        std::memcpy(h, host, bytes);
    st = upload_descriptors(ctx, bytes, s);
    if (st != RC_OK)
        return st;
    *dev_out = d;
    return RC_OK;
}

// The tile-list stream of a call whose descriptors went up in the current slot: its kernels
// start once that upload is complete.
rc::TileStream tile_stream_of(rc_context ctx)
{
    return rc::TileStream{ctx->tile_stream, ctx->desc[ctx->desc_next].uploaded, ctx->tiles_done};
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
        const auto tuned = ctx->fft_levels.find(n);
        hipError_t e = tuned != ctx->fft_levels.end() ? rc::build_fft_plan_levels(n, tuned->second, plan)
                                                       : rc::build_fft_plan(n, plan, ctx->allocs);
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

// K2 / E = e^2 / (8 pi^2 m_e eps0) (Eq 3, App. A) in long double, from the decimal constants.
long double k2_per_tec_ld()
{
    const long double e = 1.602176634e-19L, me = 9.1093837139e-31L, eps0 = 8.8541878188e-12L;
    const long double pi = 3.141592653589793238462643383279502884L;
    return e * e / (8.0L * pi * pi * me * eps0);
}

// The quarter-turn numerator s * 8 K2 / c of Eq (15)/(16) (see PhaseNum) for a pulse of n
// samples at fs with this carrier.  Its 64-bit significand keeps the phase of the bin nearest
// 0 Hz (up to ~1e12 rad with a carrier below fs/2) within ~1e-7 rad.
PhaseNum phase_numerator(double tec, int32_t direction, double fs, double carrier, int64_t n)
{
    const long double s = (direction == RC_DISTORT) ? 1.0L : -1.0L;
    const long double c4 = s * 8.0L * k2_per_tec_ld() * (long double)tec / (long double)rc::kC;
    PhaseNum P{(double)c4, 0.0, 0};
    P.lo = (double)(c4 - (long double)P.hi);
    if (P.hi == 0.0)
        return P;
    // The bin frequencies carrier + fs kk / n, kk in [-(n/2), (n-1)/2], increase with kk; the
    // smallest nonzero |f| sits at an end or next to the zero crossing.
    const int64_t lo = -(n / 2), hi = (n - 1) / 2;
    auto f_at = [&](int64_t kk) { return (long double)carrier + (long double)fs * (long double)kk / (long double)n; };
    long double fmin;
    if (f_at(lo) > 0.0L) {
        fmin = f_at(lo);
    } else if (f_at(hi) < 0.0L) {
        fmin = -f_at(hi);
    } else {
        const long double k0 = std::floor(-(long double)carrier * (long double)n / (long double)fs);
        fmin = INFINITY;
        for (int d = -1; d <= 2; ++d) {
            const long double kq = std::min(std::max(k0 + d, (long double)lo), (long double)hi);
            const long double f = std::fabs(f_at((int64_t)kq));
            if (f > 0.0L)
                fmin = std::min(fmin, f);
        }
    }
    P.xprec = std::fabs(c4) > std::ldexp(1.0L, 26) * fmin;
    return P;
}

rc::Profiler *prof_of(rc_context ctx) { return ctx->prof.on ? &ctx->prof : nullptr; }

// A JSON value, for the tuning file: objects keep their keys in order.
struct Json {
    enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
    double num = 0.0;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;
};

// Recursive-descent JSON reader (RFC 8259 grammar; \u escapes kept only for ASCII).
struct JsonReader {
    const std::string &t;
    size_t i = 0;
    std::string err;
    explicit JsonReader(const std::string &text) : t(text) {}
    void ws()
    {
        while (i < t.size() && (t[i] == ' ' || t[i] == '\t' || t[i] == '\n' || t[i] == '\r'))
            ++i;
    }
    bool fail_at(const char *what)
    {
        if (err.empty())
            err = std::string(what) + " at byte " + std::to_string(i);
        return false;
    }
    bool lit(const char *w)
    {
        const size_t n = std::strlen(w);
        if (t.compare(i, n, w) != 0)
            return fail_at("unexpected token");
        i += n;
        return true;
    }
    bool str(std::string &out)
    {
        if (i >= t.size() || t[i] != '"')
            return fail_at("expected a string");
        ++i;
        out.clear();
        while (i < t.size() && t[i] != '"') {
            char c = t[i++];
            if (c == '\\') {
                if (i >= t.size())
                    return fail_at("bad escape");
                const char e = t[i++];
                switch (e) {
                case 'n': c = '\n'; break;
                case 't': c = '\t'; break;
                case 'r': c = '\r'; break;
                case 'b': c = '\b'; break;
                case 'f': c = '\f'; break;
                case 'u': {
                    if (i + 4 > t.size())
                        return fail_at("bad escape");
                    c = (char)std::strtol(t.substr(i, 4).c_str(), nullptr, 16);
                    i += 4;
                    break;
                }
                default: c = e;
                }
            }
            out.push_back(c);
        }
        if (i >= t.size())
            return fail_at("unterminated string");
        ++i;
        return true;
    }
    bool value(Json &v, int depth)
    {
        if (depth > 64)
            return fail_at("nesting too deep");
        ws();
        if (i >= t.size())
            return fail_at("unexpected end");
        const char c = t[i];
        if (c == '{') {
            v.kind = Json::Object;
            ++i;
            ws();
            if (i < t.size() && t[i] == '}') {
                ++i;
                return true;
            }
            for (;;) {
                ws();
                std::string key;
                if (!str(key))
                    return false;
                ws();
                if (i >= t.size() || t[i] != ':')
                    return fail_at("expected ':'");
                ++i;
                Json item;
                if (!value(item, depth + 1))
                    return false;
                v.obj.emplace_back(std::move(key), std::move(item));
                ws();
                if (i < t.size() && t[i] == ',') {
                    ++i;
                    continue;
                }
                if (i < t.size() && t[i] == '}') {
                    ++i;
                    return true;
                }
                return fail_at("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v.kind = Json::Array;
            ++i;
            ws();
            if (i < t.size() && t[i] == ']') {
                ++i;
                return true;
            }
            for (;;) {
                Json item;
                if (!value(item, depth + 1))
                    return false;
                v.arr.push_back(std::move(item));
                ws();
                if (i < t.size() && t[i] == ',') {
                    ++i;
                    continue;
                }
                if (i < t.size() && t[i] == ']') {
                    ++i;
                    return true;
                }
                return fail_at("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = Json::String;
            return str(v.str);
        }
        if (c == 't') {
            v.kind = Json::Bool;
            v.num = 1.0;
            return lit("true");
        }
        if (c == 'f') {
            v.kind = Json::Bool;
            return lit("false");
        }
        if (c == 'n') {
            v.kind = Json::Null;
            return lit("null");
        }
        char *end = nullptr;
        v.num = std::strtod(t.c_str() + i, &end);
        if (end == t.c_str() + i)
            return fail_at("expected a value");
        v.kind = Json::Number;
        i = (size_t)(end - t.c_str());
        return true;
    }
};

bool parse_json(const std::string &text, Json &out, std::string &err)
{
    JsonReader r(text);
    if (!r.value(out, 0)) {
        err = r.err;
        return false;
    }
    r.ws();
    if (r.i != text.size()) {
        err = "trailing characters at byte " + std::to_string(r.i);
        return false;
    }
    return true;
}

// Workgroups per CU of the matrix-core resampler's persistent grid (0: occupancy maximum).
int sinc_grid(rc_context ctx, int half_width) { return ctx->sinc_wg_per_cu[half_width == 128 ? 1 : 0]; }

// Workspace of correct_ionosphere_noalloc: Bluestein's convolution buffer and chirp spectrum,
// 2 M complex values for a length n that is not a power of two (M the power of two >= 2n - 1),
// so M <= 2^21 and n <= 2^20.  Each device holds its own copy for the life of the process.
// Host code never takes this array's address directly: its device address comes from
// hipGetSymbolAddress, once per device with that device current (scratch_on_device).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
__device__ __align__(256) float2 scratch[kStaticScratchBytes / sizeof(float2)];

std::mutex g_scratch_mu;
constexpr int kMaxScratchDevices = 64;
float2 *g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the current device (which must be `device`).
hipError_t scratch_on_device(int device, float2 **out)
{
    if (device < 0 || device >= kMaxScratchDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[device] = static_cast<float2 *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Argument checks shared by correct_ionosphere and correct_ionosphere_noalloc.
rc_status check_iono_args(rc_context ctx, const rc_c64 *x, const rc_c64 *y, int64_t n, double fs_hz,
                          double carrier_hz, double tec_el_per_m2, int32_t direction)
{
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
    return RC_OK;
}

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
    return (double)k2_per_tec_ld();
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
    for (auto &slot : ctx->desc) {
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&slot.uploaded, hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&ctx->tile_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&ctx->tiles_done, hipEventDisableTiming);
    if (e == hipSuccess)
        e = scratch_on_device(hip_device, &ctx->static_scratch);
    if (e == hipSuccess) {
        // tuning chosen by the autotuner, when the environment names a file
        const char *tune = std::getenv("RC_TUNE_FILE");
        if (tune && *tune && rc_load_tuning(ctx, tune) != RC_OK) {
            std::fprintf(stderr, "rc_create: %s\n", ctx->last_error.c_str());
            (void)rc_destroy(ctx);
            return RC_ERR_INVALID_ARG;
        }
    }
    if (e != hipSuccess) {
        if (ctx->tiles_done)
            (void)hipEventDestroy(ctx->tiles_done);
        if (ctx->tile_stream)
            (void)hipStreamDestroy(ctx->tile_stream);
        if (ctx->copy_stream)
            (void)hipStreamDestroy(ctx->copy_stream);
        for (auto &slot : ctx->desc) {
            if (slot.done)
                (void)hipEventDestroy(slot.done);
            if (slot.uploaded)
                (void)hipEventDestroy(slot.uploaded);
        }
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
            if (slot.uploaded)
                (void)hipEventDestroy(slot.uploaded);
        }
        if (ctx->copy_stream)
            (void)hipStreamDestroy(ctx->copy_stream);
        if (ctx->tile_stream)
            (void)hipStreamDestroy(ctx->tile_stream);
        if (ctx->tiles_done)
            (void)hipEventDestroy(ctx->tiles_done);
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
        const int wpc = sinc_grid(ctx, k->half_width);
        if (!rc::sinc_mfma_uses_list(k->half_width, ntiles, wpc)) {
            e = rc::launch_sinc_mfma(nullptr, &job, 1, n_out, ntiles, nullptr, k->half_width, table, s,
                                     prof_of(ctx), nullptr, rc::TileListMode::BuildAndRun, wpc);
            break;
        }
        // a long pulse: the job descriptor and the tile list go to a staging slot
        const void *dev = nullptr;
        ts = stage_descriptors(ctx, &job, sizeof job, rc::sinc_mfma_work_bytes(ntiles), s, &dev);
        if (ts != RC_OK)
            return ts;
        char *devc = static_cast<char *>(const_cast<void *>(dev));
        const rc::TileStream tls = tile_stream_of(ctx);
        e = rc::launch_sinc_mfma(reinterpret_cast<const SincJob *>(devc), nullptr, 1, n_out, ntiles, devc + 256,
                                 k->half_width, table, s, prof_of(ctx), &tls, rc::TileListMode::BuildAndRun, wpc);
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
    rc_status vs = check_iono_args(ctx, x, y, n, fs_hz, carrier_hz, tec_el_per_m2, direction);
    if (vs != RC_OK)
        return vs;
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PhaseNum phase = phase_numerator(tec_el_per_m2, direction, fs_hz, carrier_hz, n);
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
        const rc::BluesteinJob jb{xf, yf, static_cast<float2 *>(const_cast<void *>(dev)), n, phase, carrier_hz, fs_hz,
                                  nullptr};
        e = rc::launch_iono_bluestein(*plan, ctx->tw4096, nullptr, nullptr, jb, 1, n, s, prof_of(ctx));
        st = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && st != RC_OK)
            return st;
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_ionosphere launch");
    return RC_OK;
}

rc_status correct_ionosphere_noalloc(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n, double fs_hz,
                                     double carrier_hz, double tec_el_per_m2, int32_t direction, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status vs = check_iono_args(ctx, x, y, n, fs_hz, carrier_hz, tec_el_per_m2, direction);
    if (vs != RC_OK)
        return vs;
    const bool pow2 = is_pow2(n);
    if (!pow2 && rc::bluestein_work_bytes(n) > kStaticScratchBytes)
        return fail(ctx, RC_ERR_UNSUPPORTED,
                    "correct_ionosphere_noalloc: a length that is not a power of two must be at most 2^20 "
                    "(its Bluestein workspace exceeds the static 32 MiB)");
    if (!ctx->static_scratch)
        return fail(ctx, RC_ERR_DEVICE, "the static workspace has no device address");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PhaseNum phase = phase_numerator(tec_el_per_m2, direction, fs_hz, carrier_hz, n);
    const float2 *xf = reinterpret_cast<const float2 *>(x);
    float2 *yf = reinterpret_cast<float2 *>(y);
    // the plan is rebuilt here rather than taken from (and inserted into) the context's cache,
    // with the context's tuned split if it has one; building one only fills the struct
    FftPlan plan;
    std::vector<void *> no_allocs;
    const int64_t pn = iono_plan_length(n);
    const auto tuned = ctx->fft_levels.find(pn);
    hipError_t e = tuned != ctx->fft_levels.end() ? rc::build_fft_plan_levels(pn, tuned->second, plan)
                                                   : rc::build_fft_plan(pn, plan, no_allocs);
    if (e != hipSuccess)
        return fail(ctx, RC_ERR_UNSUPPORTED, "transform length not supported");
    if (pow2) {
        const IonoJob job{xf, yf, phase, carrier_hz, fs_hz, nullptr};
        e = rc::launch_iono(plan, ctx->tw4096, nullptr, &job, 1, s, nullptr);
    } else {
        const rc::BluesteinJob jb{xf, yf, ctx->static_scratch, n, phase, carrier_hz, fs_hz, nullptr};
        e = rc::launch_iono_bluestein(plan, ctx->tw4096, nullptr, nullptr, jb, 1, n, s, nullptr);
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_ionosphere_noalloc launch");
    return RC_OK;
}

// --- the paper's other resampling methods ---------------------------------------------------

// Checks shared by the baseline resamplers: pointers, lengths, fs and alpha.
rc_status check_resample_args(rc_context ctx, const rc_c64 *x, int64_t n_in, const rc_c64 *y, int64_t n_out,
                              double fs_hz, double alpha)
{
    if (!x || !y)
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL sample pointer");
    if (n_in <= 0 || n_out <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "n_in and n_out must be > 0");
    if (!(std::isfinite(fs_hz) && fs_hz > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "fs_hz must be finite and > 0");
    if (!(std::isfinite(alpha) && alpha > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, "alpha must be finite and > 0");
    return RC_OK;
}

rc_status correct_doppler_paper(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y, int64_t n_out,
                                double fs_hz, double alpha, int32_t n_window, int32_t variant, int32_t lut_size,
                                int32_t blocks, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_resample_args(ctx, x, n_in, y, n_out, fs_hz, alpha);
    if (st != RC_OK)
        return st;
    if (overlaps(x, n_in * 8, y, n_out * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    if (n_window < 1 || (n_window & 1) == 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "n_window must be odd and >= 1");
    if (variant != RC_PAPER_DIRECT && variant != RC_PAPER_TILED && variant != RC_PAPER_LUT)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown variant");
    if (variant == RC_PAPER_LUT && (lut_size < 2 || lut_size > 16384))
        return fail(ctx, RC_ERR_INVALID_ARG, "lut_size must be in [2, 16384]");
    if (blocks < 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "blocks must be >= 0");
    const int h = (n_window - 1) / 2;
    if (variant == RC_PAPER_TILED && (alpha > 1e6 || rc::paper_tiled_lds_bytes(alpha, h) > 65536))
        return fail(ctx, RC_ERR_UNSUPPORTED, "the tiled kernel's input span exceeds 64 KiB of LDS");
    DeviceGuard g(ctx->device);
    rc::PaperArgs a{reinterpret_cast<const float2 *>(x), reinterpret_cast<float2 *>(y), n_in, n_out, alpha, h,
                    lut_size, 0.0, 0.0};
    if (variant == RC_PAPER_LUT) {
        const double u_max = (double)h + 0.5;
        a.dx = u_max / (double)(lut_size - 1);
        a.inv_dx = (double)(lut_size - 1) / u_max;
    }
    const hipError_t e = rc::launch_paper_sinc(a, variant, blocks, static_cast<hipStream_t>(stream), prof_of(ctx));
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_doppler_paper launch");
    return RC_OK;
}

rc_status correct_doppler_linear(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y, int64_t n_out,
                                 double fs_hz, double alpha, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_resample_args(ctx, x, n_in, y, n_out, fs_hz, alpha);
    if (st != RC_OK)
        return st;
    if (overlaps(x, n_in * 8, y, n_out * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    DeviceGuard g(ctx->device);
    const hipError_t e = rc::launch_linear(reinterpret_cast<const float2 *>(x), n_in, reinterpret_cast<float2 *>(y),
                                           n_out, alpha, static_cast<hipStream_t>(stream), prof_of(ctx));
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_doppler_linear launch");
    return RC_OK;
}

rc_status correct_doppler_tone(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n, double fs_hz, double alpha,
                               double f_ref_hz, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_resample_args(ctx, x, n, y, n, fs_hz, alpha);
    if (st != RC_OK)
        return st;
    if (!std::isfinite(f_ref_hz))
        return fail(ctx, RC_ERR_INVALID_ARG, "f_ref_hz must be finite");
    if (x != y && overlaps(x, n * 8, y, n * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y partially overlap");
    DeviceGuard g(ctx->device);
    const double nu = (alpha - 1.0) * f_ref_hz / fs_hz;
    const hipError_t e = rc::launch_tone(reinterpret_cast<const float2 *>(x), reinterpret_cast<float2 *>(y), n, nu,
                                         static_cast<hipStream_t>(stream), prof_of(ctx));
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_doppler_tone launch");
    return RC_OK;
}

int64_t rc_pq_length(int64_t n_in, double alpha)
{
    if (n_in < 1 || !(std::isfinite(alpha) && alpha > 0.0))
        return 0;
    const double d = ((double)n_in - (double)n_in / alpha) / 2.0;
    return n_in - 2 * (int64_t)std::llround(d);
}

rc_status correct_doppler_fft_pq(rc_context ctx, const rc_c64 *x, int64_t n_in, rc_c64 *y, int64_t n_out,
                                 double fs_hz, double alpha, double f_ref_hz, int32_t with_tone, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_resample_args(ctx, x, n_in, y, n_out, fs_hz, alpha);
    if (st != RC_OK)
        return st;
    if (!std::isfinite(f_ref_hz))
        return fail(ctx, RC_ERR_INVALID_ARG, "f_ref_hz must be finite");
    if (overlaps(x, n_in * 8, y, n_out * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    const int64_t ni = rc_pq_length(n_in, alpha);
    const int64_t kMaxPq = int64_t(1) << 23;
    if (n_in < 2 || ni < 2 || n_in > kMaxPq || ni > kMaxPq)
        return fail(ctx, RC_ERR_UNSUPPORTED, "FFT P/Q needs 2 <= n_in and the resampled length <= 2^23");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc::PqArgs a{reinterpret_cast<const float2 *>(x), reinterpret_cast<float2 *>(y), n_in, ni, n_out,
                 nullptr, nullptr, nullptr, with_tone != 0, 0.0};
    if (with_tone) {
        const double a_eff = (double)n_in / (double)ni;
        a.nu = (alpha / a_eff - 1.0) * (a_eff * f_ref_hz) / fs_hz;
    }
    const FftPlan *plan_in = nullptr, *plan_out = nullptr;
    hipError_t e;
    if (ni == n_in) {
        e = rc::launch_pq(a, FftPlan{}, FftPlan{}, ctx->tw4096, s, prof_of(ctx));
    } else {
        st = get_plan(ctx, rc::bluestein_m(n_in), &plan_in);
        if (st == RC_OK)
            st = get_plan(ctx, rc::bluestein_m(ni), &plan_out);
        if (st != RC_OK)
            return st;
        // workspace: X, then Y, then the larger Bluestein buffer, each 256-byte aligned
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t bx = al((size_t)n_in * 8), by = al((size_t)ni * 8);
        const size_t bw = std::max(rc::bluestein_work_bytes(n_in), rc::bluestein_work_bytes(ni));
        const void *dev = nullptr;
        st = stage_descriptors(ctx, nullptr, 0, bx + by + bw, s, &dev);
        if (st != RC_OK)
            return st;
        char *w = static_cast<char *>(const_cast<void *>(dev));
        a.X = reinterpret_cast<float2 *>(w);
        a.Y = reinterpret_cast<float2 *>(w + bx);
        a.work = reinterpret_cast<float2 *>(w + bx + by);
        e = rc::launch_pq(a, *plan_in, *plan_out, ctx->tw4096, s, prof_of(ctx));
        st = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && st != RC_OK)
            return st;
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "correct_doppler_fft_pq launch");
    return RC_OK;
}

rc_status replica_spectrum(rc_context ctx, const rc_c64 *replica, int64_t n_rep, int64_t n, rc_c64 *spec,
                           void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (!replica || !spec)
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL sample pointer");
    if (n <= 0 || n_rep <= 0 || n_rep > n)
        return fail(ctx, RC_ERR_INVALID_ARG, "need 1 <= n_rep <= n");
    if (overlaps(replica, n_rep * 8, spec, n * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "replica and spectrum overlap");
    if (n > kMaxIonoLength)
        return fail(ctx, RC_ERR_UNSUPPORTED, "n above 2^24 (power of two) or 2^23 (other lengths)");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FftPlan *plan = nullptr;
    rc_status st = get_plan(ctx, iono_plan_length(n), &plan);
    if (st != RC_OK)
        return st;
    float2 *sp = reinterpret_cast<float2 *>(spec);
    hipError_t e = rc::launch_pad(reinterpret_cast<const float2 *>(replica), n_rep, sp, n, s);
    if (e == hipSuccess && is_pow2(n)) {
        // the transform's native bin order, which the row pass of compress_pulse multiplies in
        const IonoJob jb{sp, sp, PhaseNum{}, 0.0, 0.0, nullptr, 0};
        e = rc::launch_fft_forward(*plan, ctx->tw4096, nullptr, &jb, 1, s, prof_of(ctx));
    } else if (e == hipSuccess) {
        // natural bin order, which Bluestein's middle step of compress_pulse multiplies in
        const void *dev = nullptr;
        st = stage_descriptors(ctx, nullptr, 0, rc::bluestein_work_bytes(n), s, &dev);
        if (st != RC_OK)
            return st;
        const rc::BluesteinJob jb{sp, sp, static_cast<float2 *>(const_cast<void *>(dev)), n, PhaseNum{}, 0.0, 0.0, nullptr};
        e = rc::launch_bluestein_forward(*plan, ctx->tw4096, jb, s, prof_of(ctx));
        st = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && st != RC_OK)
            return st;
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "replica_spectrum launch");
    return RC_OK;
}

rc_status compress_pulse(rc_context ctx, const rc_c64 *x, rc_c64 *y, int64_t n, const rc_c64 *spec, double fs_hz,
                         double carrier_hz, double tec_el_per_m2, int32_t direction, void *stream)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (!x || !y || !spec)
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
    if (overlaps(spec, n * 8, y, n * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "the spectrum overlaps y");
    if (n > kMaxIonoLength)
        return fail(ctx, RC_ERR_UNSUPPORTED, "n above 2^24 (power of two) or 2^23 (other lengths)");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const FftPlan *plan = nullptr;
    rc_status st = get_plan(ctx, iono_plan_length(n), &plan);
    if (st != RC_OK)
        return st;
    const float2 *xf = reinterpret_cast<const float2 *>(x);
    float2 *yf = reinterpret_cast<float2 *>(y);
    const float2 *sp = reinterpret_cast<const float2 *>(spec);
    const PhaseNum phase = phase_numerator(tec_el_per_m2, direction, fs_hz, carrier_hz, n);
    hipError_t e;
    if (is_pow2(n)) {
        const IonoJob job{xf, yf, phase, carrier_hz, fs_hz, sp, 1};
        e = rc::launch_iono(*plan, ctx->tw4096, nullptr, &job, 1, s, prof_of(ctx), rc::kRowTablePhase);
    } else {
        const void *dev = nullptr;
        st = stage_descriptors(ctx, nullptr, 0, rc::bluestein_work_bytes(n), s, &dev);
        if (st != RC_OK)
            return st;
        const rc::BluesteinJob jb{xf, yf, static_cast<float2 *>(const_cast<void *>(dev)), n, phase, carrier_hz,
                                  fs_hz, sp};
        e = rc::launch_iono_bluestein(*plan, ctx->tw4096, nullptr, nullptr, jb, 1, n, s, prof_of(ctx));
        st = mark_descriptors_used(ctx, s);
        if (e == hipSuccess && st != RC_OK)
            return st;
    }
    if (e != hipSuccess)
        return device_fail(ctx, e, "compress_pulse launch");
    return RC_OK;
}

namespace {

// Workspace cap of one Bluestein launch sequence in a batch (at least one pulse runs).
constexpr size_t kBluesteinChunkBytes = size_t(256) << 20;

// One pulse of work, with device pointers (a packed-batch entry, a server request, a bank row).
struct PulseWork {
    const float2 *x;
    float2 *y;
    int64_t n_in, n_out;
    double fs_hz, alpha, tec, carrier;
    uint32_t flags;
    int32_t direction;
};

rc_status validate_pulse(rc_context ctx, const PulseWork &p, const std::string &at)
{
    if (p.n_in <= 0 || p.n_out <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, at + "n_in and n_out must be > 0");
    if ((p.flags & ~(uint32_t)(RC_DO_DOPPLER | RC_DO_IONO)) != 0)
        return fail(ctx, RC_ERR_INVALID_ARG, at + "unknown flag bits");
    if (!(std::isfinite(p.fs_hz) && p.fs_hz > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, at + "fs_hz must be finite and > 0");
    if ((p.flags & RC_DO_DOPPLER) && !(std::isfinite(p.alpha) && p.alpha > 0.0))
        return fail(ctx, RC_ERR_INVALID_ARG, at + "alpha must be finite and > 0");
    if (!(p.flags & RC_DO_DOPPLER) && p.n_out != p.n_in)
        return fail(ctx, RC_ERR_INVALID_ARG, at + "n_out must equal n_in without RC_DO_DOPPLER");
    if (p.flags & RC_DO_IONO) {
        if (!(std::isfinite(p.tec) && p.tec >= 0.0) || !std::isfinite(p.carrier))
            return fail(ctx, RC_ERR_INVALID_ARG, at + "tec must be finite and >= 0, carrier finite");
        if (p.direction != RC_CORRECT && p.direction != RC_DISTORT)
            return fail(ctx, RC_ERR_INVALID_ARG, at + "bad direction");
        if (p.n_out > kMaxIonoLength || (!is_pow2(p.n_out) && 2 * p.n_out - 1 > kMaxIonoLength))
            return fail(ctx, RC_ERR_UNSUPPORTED, at + "iono length above 2^24 (power of two) or 2^23 (other)");
    }
    return RC_OK;
}

rc_status run_pulses_locked(rc_context ctx, const std::vector<PulseWork> &work, const rc_sinc *k, hipStream_t s);
rc_status batch_work(rc_context ctx, const rc_c64 *x_packed, int64_t x_len, rc_c64 *y_packed, int64_t y_len,
                     const rc_pulse *pulses, int32_t count, std::vector<PulseWork> &work);

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
    std::vector<PulseWork> work;
    st = batch_work(ctx, x_packed, x_len, y_packed, y_len, pulses, count, work);
    if (st != RC_OK)
        return st;
    return run_pulses_locked(ctx, work, k, static_cast<hipStream_t>(stream));
}

// Validate a packed batch (every pulse inside its buffer, output ranges pairwise disjoint) into
// its list of pulses with device pointers.
rc_status batch_work(rc_context ctx, const rc_c64 *x_packed, int64_t x_len, rc_c64 *y_packed, int64_t y_len,
                     const rc_pulse *pulses, int32_t count, std::vector<PulseWork> &work)
{
    rc_status st = RC_OK;
    const float2 *xb = reinterpret_cast<const float2 *>(x_packed);
    float2 *yb = reinterpret_cast<float2 *>(y_packed);
    std::vector<std::pair<int64_t, int64_t>> outs;
    work.clear();
    outs.reserve((size_t)count);
    work.reserve((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const rc_pulse &p = pulses[i];
        const std::string at = "pulse " + std::to_string(i) + ": ";
        if (p.n_in <= 0 || p.n_out <= 0 || p.off_in < 0 || p.off_out < 0 || p.off_in > x_len - p.n_in ||
            p.off_out > y_len - p.n_out)
            return fail(ctx, RC_ERR_INVALID_ARG, at + "range outside its buffer");
        const PulseWork w{xb + p.off_in, yb + p.off_out, p.n_in, p.n_out, p.fs_hz, p.alpha, p.tec_el_per_m2,
                          p.carrier_hz, p.flags, p.direction};
        st = validate_pulse(ctx, w, at);
        if (st != RC_OK)
            return st;
        work.push_back(w);
        outs.emplace_back(p.off_out, p.off_out + p.n_out);
    }
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].first < outs[i - 1].second)
            return fail(ctx, RC_ERR_INVALID_ARG, "output ranges overlap");
    return RC_OK;
}

// A validated list of pulses grouped for launching: Doppler jobs by engine, ionospheric jobs by
// transform length (Bluestein ones in chunks by convolution length), plain copies for pulses with
// neither step; and the descriptor blob the launches read, uploaded as one piece.
struct BlueChunk {
    int64_t m, max_n;
    size_t first, count, off_jobs, off_ffts;
};
struct BatchPrep {
    std::vector<SincJob> mfma, fast, direct;
    int64_t mfma_max = 0, fast_max = 0, direct_max = 0, direct_taps = 0;
    std::map<int64_t, std::vector<IonoJob>> iono;           // power-of-two lengths, by length
    std::map<int64_t, std::vector<rc::BluesteinJob>> blue;  // other lengths, by convolution length
    std::vector<BlueChunk> chunks;
    std::vector<int32_t> copies;
    const void *mfma_table = nullptr;
    int64_t mfma_tiles = 0;
    size_t mfma_work = 0, bs_work = 0;
    std::vector<char> blob;  // [mfma | fast | direct | iono groups | Bluestein chunks]
    size_t off_mfma = 0, off_fast = 0, off_direct = 0;
    std::vector<size_t> off_iono;
    // device bytes after the descriptors: [tile list][Bluestein], each region 256-byte aligned
    static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }
    size_t extra() const { return mfma_work || bs_work ? al(mfma_work) + bs_work : 0; }
    size_t device_bytes() const { return extra() ? al(blob.size()) + extra() : blob.size(); }
};

rc_status prepare_batch(rc_context ctx, const std::vector<PulseWork> &work, const rc_sinc *k, BatchPrep &bp)
{
    rc_status st = RC_OK;
    const int32_t count = (int32_t)work.size();
    for (int32_t i = 0; i < count; ++i) {
        const PulseWork &p = work[(size_t)i];
        if (p.flags & RC_DO_DOPPLER) {
            const SincJob j{p.x, p.y, p.n_in, p.n_out, p.alpha, 0};
            const SincPath path = sinc_path(ctx, p.alpha, *k);
            if (path == SincPath::Mfma) {
                bp.mfma.push_back(j);
                bp.mfma_max = std::max(bp.mfma_max, p.n_out);
            } else if (path == SincPath::Fast) {
                bp.fast.push_back(j);
                bp.fast_max = std::max(bp.fast_max, p.n_out);
            } else {
                bp.direct.push_back(j);
                bp.direct_max = std::max(bp.direct_max, p.n_out);
                bp.direct_taps = std::max(bp.direct_taps, taps_per_output(*k, p.n_in));
            }
        } else if (!(p.flags & RC_DO_IONO)) {
            bp.copies.push_back(i);
        }
        if (p.flags & RC_DO_IONO) {
            const float2 *src = (p.flags & RC_DO_DOPPLER) ? p.y : p.x;
            const PhaseNum ph = phase_numerator(p.tec, p.direction, p.fs_hz, p.carrier, p.n_out);
            if (is_pow2(p.n_out))
                bp.iono[p.n_out].push_back(IonoJob{src, p.y, ph, p.carrier, p.fs_hz, nullptr});
            else
                bp.blue[rc::bluestein_m(p.n_out)].push_back(
                    rc::BluesteinJob{src, p.y, nullptr, p.n_out, ph, p.carrier, p.fs_hz, nullptr});
        }
    }
    if (bp.mfma.size() > 65535 || bp.fast.size() > 65535 || bp.direct.size() > 65535)
        return fail(ctx, RC_ERR_UNSUPPORTED, "more than 65535 pulses of one kind in a batch");
    for (auto &kv : bp.iono) {
        const FftPlan *plan = nullptr;
        st = get_plan(ctx, kv.first, &plan);
        if (st != RC_OK)
            return st;
    }
    // Bluestein pulses of one convolution length run in chunks of one launch sequence each; a
    // chunk's pulses have workspaces side by side in one region (at most kBluesteinChunkBytes,
    // or one pulse), reused by the next chunk in stream order.
    for (auto &kv : bp.blue) {
        const FftPlan *plan = nullptr;
        st = get_plan(ctx, kv.first, &plan);
        if (st != RC_OK)
            return st;
        const size_t per = rc::bluestein_work_bytes(kv.second[0].n);  // 2 m complex values
        const size_t chunk = ctx->bluestein_chunk > 0 ? (size_t)ctx->bluestein_chunk : kBluesteinChunkBytes;
        const size_t cap = std::max<size_t>(1, std::min<size_t>(65535, chunk / per));
        for (size_t b = 0; b < kv.second.size(); b += cap) {
            const size_t cnt = std::min(cap, kv.second.size() - b);
            int64_t mx = 0;
            for (size_t i = b; i < b + cnt; ++i)
                mx = std::max(mx, kv.second[i].n);
            bp.chunks.push_back(BlueChunk{kv.first, mx, b, cnt, 0, 0});
            bp.bs_work = std::max(bp.bs_work, cnt * per);
        }
    }
    if (!bp.mfma.empty()) {
        st = get_mfma_table(ctx, *k, &bp.mfma_table);
        if (st != RC_OK)
            return st;
        for (SincJob &j : bp.mfma) {
            j.tile0 = bp.mfma_tiles;
            bp.mfma_tiles += (j.n_out + rc::kSincMfmaTile - 1) / rc::kSincMfmaTile;
        }
        if (bp.mfma_tiles > 0x7fffffff)
            return fail(ctx, RC_ERR_UNSUPPORTED, "more than 2^31 - 1 matrix-core tiles in a batch");
        if (rc::sinc_mfma_uses_list(k->half_width, bp.mfma_tiles, sinc_grid(ctx, k->half_width)))
            bp.mfma_work = rc::sinc_mfma_work_bytes(bp.mfma_tiles);
    }
    auto append = [&](const void *p, size_t bytes) {
        const size_t off = (bp.blob.size() + 15) & ~(size_t)15;
        bp.blob.resize(off + bytes);
        std::memcpy(bp.blob.data() + off, p, bytes);
        return off;
    };
    bp.off_mfma = bp.mfma.empty() ? 0 : append(bp.mfma.data(), bp.mfma.size() * sizeof(SincJob));
    bp.off_fast = bp.fast.empty() ? 0 : append(bp.fast.data(), bp.fast.size() * sizeof(SincJob));
    bp.off_direct = bp.direct.empty() ? 0 : append(bp.direct.data(), bp.direct.size() * sizeof(SincJob));
    for (auto &kv : bp.iono)
        bp.off_iono.push_back(append(kv.second.data(), kv.second.size() * sizeof(IonoJob)));
    // per Bluestein chunk: its jobs, then 2 x count FFT jobs (chirp transforms, convolutions);
    // their workspace pointers are filled in once the device address is known
    for (BlueChunk &c : bp.chunks) {
        c.off_jobs = append(bp.blue[c.m].data() + c.first, c.count * sizeof(rc::BluesteinJob));
        const std::vector<IonoJob> blank(2 * c.count);
        c.off_ffts = append(blank.data(), blank.size() * sizeof(IonoJob));
    }
    return RC_OK;
}

// The Bluestein workspace pointers of the blob, for a device copy of it at devc.
void point_bluestein_work(BatchPrep &bp, char *devc)
{
    float2 *bw = reinterpret_cast<float2 *>(devc + BatchPrep::al(bp.blob.size()) + BatchPrep::al(bp.mfma_work));
    for (const BlueChunk &c : bp.chunks) {
        auto *jobs = reinterpret_cast<rc::BluesteinJob *>(bp.blob.data() + c.off_jobs);
        auto *ffts = reinterpret_cast<IonoJob *>(bp.blob.data() + c.off_ffts);
        for (size_t q = 0; q < c.count; ++q) {
            float2 *a = bw + (size_t)q * 2 * c.m, *b = a + c.m;
            jobs[q].a = a;
            ffts[q] = IonoJob{b, b, PhaseNum{}, 0.0, 0.0, nullptr};
            ffts[c.count + q] = IonoJob{a, a, PhaseNum{}, 0.0, 0.0, b};
        }
    }
}

// Enqueue the batch's work on s, its descriptors (and workspace) at devc on the device.
rc_status enqueue_batch(rc_context ctx, const BatchPrep &bp, const std::vector<PulseWork> &work, const rc_sinc *k,
                        char *devc, hipStream_t s, rc::Profiler *prof, const rc::TileStream *tls,
                        rc::TileListMode mode)
{
    char *wbase = bp.extra() ? devc + BatchPrep::al(bp.blob.size()) : nullptr;
    void *tile_work = bp.mfma_work ? wbase : nullptr;
    hipError_t e = hipSuccess;
    if (mode == rc::TileListMode::BuildOnly) {
        if (!bp.mfma.empty())
            e = rc::launch_sinc_mfma(reinterpret_cast<const SincJob *>(devc + bp.off_mfma), nullptr,
                                     (int)bp.mfma.size(), bp.mfma_max, bp.mfma_tiles, tile_work, k->half_width,
                                     bp.mfma_table, s, nullptr, nullptr, mode, sinc_grid(ctx, k->half_width));
        return e == hipSuccess ? RC_OK : device_fail(ctx, e, "batch tile list");
    }
    for (int32_t i : bp.copies) {
        const PulseWork &p = work[(size_t)i];
        e = hipMemcpyAsync(p.y, p.x, (size_t)p.n_in * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return device_fail(ctx, e, "copy");
    }
    const rc::KaiserPoly kp = rc::make_kaiser_poly(k->window == RC_WIN_KAISER ? k->kaiser_beta : 0.0);
    if (!bp.mfma.empty())
        e = rc::launch_sinc_mfma(reinterpret_cast<const SincJob *>(devc + bp.off_mfma), nullptr, (int)bp.mfma.size(),
                                 bp.mfma_max, bp.mfma_tiles, tile_work, k->half_width, bp.mfma_table, s, prof, tls,
                                 mode, sinc_grid(ctx, k->half_width));
    if (e == hipSuccess && !bp.fast.empty())
        e = rc::launch_sinc_fast(reinterpret_cast<const SincJob *>(devc + bp.off_fast), nullptr, (int)bp.fast.size(),
                                 bp.fast_max, k->half_width, kp, s, prof);
    if (e == hipSuccess && !bp.direct.empty())
        e = rc::launch_sinc_direct(reinterpret_cast<const SincJob *>(devc + bp.off_direct), nullptr,
                                   (int)bp.direct.size(), bp.direct_max, *k, kp, bp.direct_taps, s, prof);
    if (e != hipSuccess)
        return device_fail(ctx, e, "batch Doppler launch");
    for (const BlueChunk &c : bp.chunks) {
        const FftPlan *plan = nullptr;
        rc_status st = get_plan(ctx, c.m, &plan);
        if (st != RC_OK)
            return st;
        e = rc::launch_iono_bluestein(*plan, ctx->tw4096, reinterpret_cast<const rc::BluesteinJob *>(devc + c.off_jobs),
                                      reinterpret_cast<const IonoJob *>(devc + c.off_ffts), rc::BluesteinJob{},
                                      (int)c.count, c.max_n, s, prof);
        if (e != hipSuccess)
            return device_fail(ctx, e, "batch ionosphere launch");
    }
    size_t gi = 0;
    for (auto &kv : bp.iono) {
        const FftPlan *plan = nullptr;
        rc_status st = get_plan(ctx, kv.first, &plan);
        if (st != RC_OK)
            return st;
        const IonoJob *jd = reinterpret_cast<const IonoJob *>(devc + bp.off_iono[gi++]);
        // at most 65535 pulses per launch keeps every grid dimension in range
        for (size_t b = 0; b < kv.second.size(); b += 65535) {
            const int nj = (int)std::min<size_t>(65535, kv.second.size() - b);
            e = rc::launch_iono(*plan, ctx->tw4096, jd + b, nullptr, nj, s, prof);
            if (e != hipSuccess)
                return device_fail(ctx, e, "batch ionosphere launch");
        }
    }
    return RC_OK;
}

// Launch a validated list of pulses on `s`, its descriptors staged through the context's ring.
rc_status run_pulses_locked(rc_context ctx, const std::vector<PulseWork> &work, const rc_sinc *k, hipStream_t s)
{
    DeviceGuard g(ctx->device);
    BatchPrep bp;
    rc_status st = prepare_batch(ctx, work, k, bp);
    if (st != RC_OK)
        return st;
    const size_t extra = bp.extra();
    char *devc = nullptr;
    if (!bp.blob.empty() || extra) {
        void *host = nullptr;
        st = reserve_descriptors(ctx, bp.blob.size(), extra, &host, &devc);
        if (st != RC_OK)
            return st;
        point_bluestein_work(bp, devc);
        if (!bp.blob.empty())
            std::memcpy(host, bp.blob.data(), bp.blob.size());
        st = upload_descriptors(ctx, bp.blob.size(), s);
        if (st != RC_OK) {
            (void)mark_descriptors_used(ctx, s);
            return st;
        }
    }
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
    } slot_mark{ctx, s, devc != nullptr};
    rc::TileStream tls{};
    if (!bp.mfma.empty())
        tls = tile_stream_of(ctx);
    st = enqueue_batch(ctx, bp, work, k, devc, s, prof_of(ctx), bp.mfma.empty() ? nullptr : &tls,
                       rc::TileListMode::BuildAndRun);
    if (st != RC_OK)
        return st;
    if (devc) {
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

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Batch plans: one batch's launch sequence captured once in a HIP graph and replayed.

struct rc_batch_plan_s {
    rc_context ctx = nullptr;
    rc_sinc k{};
    const rc_c64 *x = nullptr;
    rc_c64 *y = nullptr;
    int64_t x_len = 0, y_len = 0;
    std::vector<PulseWork> work;
    BatchPrep bp;
    char *dev = nullptr;            // descriptors, then the tile list and Bluestein workspace
    void *host = nullptr;           // pinned staging of descriptor updates
    hipEvent_t uploaded = nullptr;  // the last update's upload (the staging buffer is free after it)
    hipStream_t stream = nullptr;   // set-up and capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::mutex mu;
};

namespace {

// Two preparations launch the same graph: the same groups in the same order with the same
// lengths, tile counts, Bluestein chunks and descriptor layout, and the same plain copies.
bool same_launches(const BatchPrep &a, const BatchPrep &b, const std::vector<PulseWork> &wa,
                   const std::vector<PulseWork> &wb)
{
    auto same_jobs = [](const std::vector<SincJob> &u, const std::vector<SincJob> &v) {
        if (u.size() != v.size())
            return false;
        for (size_t i = 0; i < u.size(); ++i)
            if (u[i].n_in != v[i].n_in || u[i].n_out != v[i].n_out || u[i].tile0 != v[i].tile0)
                return false;
        return true;
    };
    if (!same_jobs(a.mfma, b.mfma) || !same_jobs(a.fast, b.fast) || !same_jobs(a.direct, b.direct))
        return false;
    if (a.mfma_max != b.mfma_max || a.fast_max != b.fast_max || a.direct_max != b.direct_max ||
        a.direct_taps != b.direct_taps || a.mfma_tiles != b.mfma_tiles || a.mfma_work != b.mfma_work ||
        a.bs_work != b.bs_work || a.mfma_table != b.mfma_table || a.blob.size() != b.blob.size())
        return false;
    if (a.iono.size() != b.iono.size() || a.chunks.size() != b.chunks.size() || a.copies != b.copies)
        return false;
    for (auto ia = a.iono.begin(), ib = b.iono.begin(); ia != a.iono.end(); ++ia, ++ib)
        if (ia->first != ib->first || ia->second.size() != ib->second.size())
            return false;
    for (size_t i = 0; i < a.chunks.size(); ++i) {
        const BlueChunk &p = a.chunks[i], &q = b.chunks[i];
        if (p.m != q.m || p.max_n != q.max_n || p.first != q.first || p.count != q.count ||
            p.off_jobs != q.off_jobs || p.off_ffts != q.off_ffts)
            return false;
    }
    for (int32_t i : a.copies)  // the graph's copy nodes hold their pointers
        if (wa[(size_t)i].x != wb[(size_t)i].x || wa[(size_t)i].y != wb[(size_t)i].y)
            return false;
    return true;
}

void free_plan(rc_batch_plan p)
{
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->uploaded)
        (void)hipEventDestroy(p->uploaded);
    if (p->stream)
        (void)hipStreamDestroy(p->stream);
    if (p->host)
        (void)hipHostFree(p->host);
    if (p->dev)
        (void)hipFree(p->dev);
    delete p;
}

}  // namespace

extern "C" {

rc_status rc_batch_plan_create(rc_context ctx, const rc_c64 *x_packed, int64_t x_len, rc_c64 *y_packed,
                               int64_t y_len, const rc_pulse *pulses, int32_t count, const rc_sinc *k,
                               rc_batch_plan *out)
{
    if (!ctx || !out)
        return RC_ERR_INVALID_ARG;
    *out = nullptr;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    rc_status st = check_sinc(ctx, k);
    if (st != RC_OK)
        return st;
    if (count <= 0 || !pulses || !x_packed || !y_packed)
        return fail(ctx, RC_ERR_INVALID_ARG, "a plan needs count >= 1 and non-NULL pointers");
    if (x_len <= 0 || y_len <= 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "buffer lengths must be > 0");
    if (overlaps(x_packed, x_len * 8, y_packed, y_len * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "input and output buffers overlap");
    rc_batch_plan p = new (std::nothrow) rc_batch_plan_s();
    if (!p)
        return RC_ERR_OUT_OF_MEMORY;
    p->ctx = ctx;
    p->k = *k;
    p->x = x_packed;
    p->y = y_packed;
    p->x_len = x_len;
    p->y_len = y_len;
    st = batch_work(ctx, x_packed, x_len, y_packed, y_len, pulses, count, p->work);
    if (st == RC_OK)
        st = prepare_batch(ctx, p->work, k, p->bp);
    if (st != RC_OK) {
        delete p;
        return st;
    }
    DeviceGuard g(ctx->device);
    auto bail = [&](hipError_t e, const char *where) {
        free_plan(p);
        return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation
                   ? fail(ctx, RC_ERR_OUT_OF_MEMORY, std::string(where) + ": out of device memory")
                   : device_fail(ctx, e, where);
    };
    const size_t bytes = p->bp.device_bytes();
    hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming);
    if (e != hipSuccess)
        return bail(e, "batch plan stream");
    if (bytes) {
        e = hipMalloc(reinterpret_cast<void **>(&p->dev), bytes);
        if (e == hipSuccess && !p->bp.blob.empty())
            e = hipHostMalloc(&p->host, p->bp.blob.size(), hipHostMallocDefault);
        if (e != hipSuccess)
            return bail(e, "batch plan workspace");
        point_bluestein_work(p->bp, p->dev);
        if (!p->bp.blob.empty()) {
            std::memcpy(p->host, p->bp.blob.data(), p->bp.blob.size());
            e = hipMemcpyAsync(p->dev, p->host, p->bp.blob.size(), hipMemcpyHostToDevice, p->stream);
            if (e == hipSuccess)
                e = hipEventRecord(p->uploaded, p->stream);
            if (e != hipSuccess)
                return bail(e, "batch plan descriptors");
        }
    }
    // the tile list depends on the descriptors only: built once here (and on updates)
    st = enqueue_batch(ctx, p->bp, p->work, &p->k, p->dev, p->stream, nullptr, nullptr, rc::TileListMode::BuildOnly);
    if (st != RC_OK) {
        free_plan(p);
        return st;
    }
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess)
        return bail(e, "batch plan set-up");
    e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return bail(e, "batch plan capture");
    st = enqueue_batch(ctx, p->bp, p->work, &p->k, p->dev, p->stream, nullptr, nullptr, rc::TileListMode::RunOnly);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->stream, &graph);
    p->graph = graph;
    if (st != RC_OK) {
        free_plan(p);
        return st;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return bail(e, "batch plan graph");
    *out = p;
    return RC_OK;
}

rc_status rc_batch_plan_launch(rc_batch_plan plan, void *stream)
{
    if (!plan)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(plan->mu);
    DeviceGuard g(plan->ctx->device);
    const hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lc(plan->ctx->mu);
        return device_fail(plan->ctx, e, "rc_batch_plan_launch");
    }
    return RC_OK;
}

rc_status rc_batch_plan_update(rc_batch_plan plan, const rc_pulse *pulses, int32_t count, void *stream)
{
    if (!plan)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lp(plan->mu);
    rc_context ctx = plan->ctx;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (count != (int32_t)plan->work.size() || !pulses)
        return fail(ctx, RC_ERR_INVALID_ARG, "an update must give the plan's number of pulses");
    std::vector<PulseWork> work;
    rc_status st = batch_work(ctx, plan->x, plan->x_len, plan->y, plan->y_len, pulses, count, work);
    if (st != RC_OK)
        return st;
    BatchPrep bp;
    st = prepare_batch(ctx, work, &plan->k, bp);
    if (st != RC_OK)
        return st;
    if (!same_launches(plan->bp, bp, plan->work, work))
        return fail(ctx, RC_ERR_UNSUPPORTED,
                    "these pulses need other launches than the plan's (lengths, flags, resampling engines, "
                    "Bluestein groups or copies differ): create a new plan");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!bp.blob.empty()) {
        point_bluestein_work(bp, plan->dev);
        e = hipEventSynchronize(plan->uploaded);  // the staging buffer's last upload has been read
        if (e == hipSuccess) {
            std::memcpy(plan->host, bp.blob.data(), bp.blob.size());
            e = hipMemcpyAsync(plan->dev, plan->host, bp.blob.size(), hipMemcpyHostToDevice, s);
        }
        if (e == hipSuccess)
            e = hipEventRecord(plan->uploaded, s);
        if (e != hipSuccess)
            return device_fail(ctx, e, "rc_batch_plan_update");
    }
    st = enqueue_batch(ctx, bp, work, &plan->k, plan->dev, s, nullptr, nullptr, rc::TileListMode::BuildOnly);
    if (st != RC_OK)
        return st;
    plan->work = std::move(work);
    plan->bp = std::move(bp);
    return RC_OK;
}

rc_status rc_batch_plan_destroy(rc_batch_plan plan)
{
    if (!plan)
        return RC_ERR_INVALID_ARG;
    {
        DeviceGuard g(plan->ctx->device);
        (void)hipDeviceSynchronize();  // no launch of the plan may still read its buffers
    }
    free_plan(plan);
    return RC_OK;
}

rc_status correct_doppler_bank(rc_context ctx, const rc_c64 *x, int64_t n, rc_c64 *y, int64_t n_out, double fs_hz,
                               const double *alphas, int32_t n_hyp, const rc_sinc *k, int32_t precision,
                               void *stream)
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
    if (precision != RC_BANK_FP16X3 && precision != RC_BANK_BF16X3 && precision != RC_BANK_FP32)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown bank precision");
    for (int32_t h = 0; h < n_hyp; ++h)
        if (!(std::isfinite(alphas[h]) && alphas[h] > 0.0))
            return fail(ctx, RC_ERR_INVALID_ARG, "hypothesis " + std::to_string(h) + ": alpha must be finite and > 0");
    if (n_out > INT64_MAX / 8 / n_hyp)
        return fail(ctx, RC_ERR_INVALID_ARG, "output size overflows");
    if (overlaps(x, n * 8, y, n_out * n_hyp * 8))
        return fail(ctx, RC_ERR_INVALID_ARG, "x and y overlap");
    const int mode = ctx->bank_engine;
    const bool farrow = mode != RC_BANK_ENGINE_PER_HYPOTHESIS && rc::farrow_eligible(*k, alphas, n_hyp);
    if (mode == RC_BANK_ENGINE_FARROW && !farrow)
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
                                          n_out, k->half_width, precision, coef, devc,
                                          devc + ((desc.size() + 255) & ~(size_t)255),
                                          s, prof_of(ctx));
    st = mark_descriptors_used(ctx, s);
    if (e != hipSuccess)
        return device_fail(ctx, e, "Doppler bank launch");
    return st;
}

// ---------------------------------------------------------------------------------------
// Serving: continuous batching of independent requests on the server's own stream.

struct rc_server_s {
    using clock = std::chrono::steady_clock;
    struct Req {
        int64_t ticket;
        PulseWork work;
        int64_t bytes;
        clock::time_point submitted;
        hipEvent_t ready;  // recorded on the request's stream at submission
    };
    struct Flight {
        hipEvent_t done;
        std::vector<Req> reqs;
        rc_status status;
    };
    struct Ticket {
        bool done = false;
        rc_status status = RC_OK;
    };
    rc_context ctx = nullptr;
    rc_sinc k{};
    int64_t budget = 0;
    int32_t max_batch = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_queue, cv_flight, cv_done;
    std::deque<Req> queue;                       // admitted, not launched
    std::deque<Flight> flights;                  // launched, not complete (stream order)
    std::unordered_map<int64_t, Ticket> tickets; // admitted, not yet waited for
    std::vector<hipEvent_t> event_pool;
    std::vector<hipEvent_t> ready_pool;          // request-ready events no request holds
    int64_t in_flight_bytes = 0;                 // admitted and not complete
    int64_t next_ticket = 1;
    bool stop = false, launcher_done = false;
    std::thread launcher, completer;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, batched_reqs = 0, samples = 0;
    std::vector<double> latency_ms;
    bool have_first = false;
    clock::time_point first_submit, last_done;
};

namespace {

// Batches a server keeps on the device at once: one running and one queued behind it.
constexpr int kServerFlights = 2;

void server_launcher(rc_server srv)
{
    for (;;) {
        std::vector<rc_server_s::Req> take;
        hipEvent_t ev = nullptr;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            // Launch when something is queued and fewer than kServerFlights batches are on the
            // device: under load the queue fills meanwhile and the next batch takes all of it
            // (up to max_batch), so the per-launch cost is shared; at light load a request
            // starts at once.
            srv->cv_queue.wait(lk, [&] {
                return (srv->stop && srv->queue.empty()) ||
                       (!srv->queue.empty() && (int)srv->flights.size() < kServerFlights);
            });
            if (srv->queue.empty()) {  // stop requested and nothing left
                srv->launcher_done = true;
                srv->cv_flight.notify_all();
                return;
            }
            while (!srv->queue.empty() && (int32_t)take.size() < srv->max_batch) {
                take.push_back(srv->queue.front());
                srv->queue.pop_front();
            }
            if (!srv->event_pool.empty()) {
                ev = srv->event_pool.back();
                srv->event_pool.pop_back();
            }
        }
        std::vector<PulseWork> work;
        work.reserve(take.size());
        for (const auto &r : take)
            work.push_back(r.work);
        rc_status st;
        {
            std::lock_guard<std::mutex> lk(srv->ctx->mu);
            srv->ctx->last_error.clear();
            DeviceGuard g(srv->ctx->device);
            st = RC_OK;
            for (const auto &r : take)
                if (hipStreamWaitEvent(srv->stream, r.ready, 0) != hipSuccess)
                    st = RC_ERR_DEVICE;
            if (st == RC_OK)
                st = run_pulses_locked(srv->ctx, work, &srv->k, srv->stream);
            if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
                ev = nullptr;
            if (ev && hipEventRecord(ev, srv->stream) != hipSuccess)
                st = RC_ERR_DEVICE;
            if (!ev)
                st = RC_ERR_DEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->flights.push_back({ev, std::move(take), st});
            srv->batches += 1;
            srv->batched_reqs += (int64_t)srv->flights.back().reqs.size();
        }
        srv->cv_flight.notify_all();
    }
}

void server_completer(rc_server srv)
{
    for (;;) {
        rc_server_s::Flight f;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_flight.wait(lk, [&] { return !srv->flights.empty() || srv->launcher_done; });
            if (srv->flights.empty())
                return;  // the launcher has stopped and every batch is complete
            f = srv->flights.front();
        }
        rc_status st = f.status;
        if (f.done) {
            DeviceGuard g(srv->ctx->device);
            if (hipEventSynchronize(f.done) != hipSuccess && st == RC_OK)
                st = RC_ERR_DEVICE;
        }
        const auto now = rc_server_s::clock::now();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->flights.pop_front();
            for (const auto &r : f.reqs) {
                auto it = srv->tickets.find(r.ticket);
                if (it != srv->tickets.end()) {
                    it->second.done = true;
                    it->second.status = st;
                }
                srv->in_flight_bytes -= r.bytes;
                srv->ready_pool.push_back(r.ready);
                srv->completed += 1;
                srv->samples += r.work.n_out;
                srv->latency_ms.push_back(std::chrono::duration<double, std::milli>(now - r.submitted).count());
            }
            srv->last_done = now;
            if (f.done)
                srv->event_pool.push_back(f.done);
        }
        srv->cv_done.notify_all();
        srv->cv_queue.notify_all();  // a flight slot is free
    }
}

// Bytes a request holds while admitted: its input and output, and an upper bound of its share
// of a batch's device workspace, so that the workspace of the batches in flight never exceeds
// the server's budget: the Bluestein buffers of a length that is not a power of two
// (bluestein_work_bytes), the matrix-core tile list of a Doppler pulse on that path, and 1 KiB
// for its descriptors and the workspace regions' alignment.
int64_t request_bytes(rc_context ctx, const PulseWork &w, const rc_sinc &k)
{
    int64_t b = 8 * (w.n_in + w.n_out) + 1024;
    if ((w.flags & RC_DO_IONO) && !is_pow2(w.n_out))
        b += (int64_t)rc::bluestein_work_bytes(w.n_out);
    if ((w.flags & RC_DO_DOPPLER) && sinc_path(ctx, w.alpha, k) == SincPath::Mfma)
        b += (int64_t)rc::sinc_mfma_work_bytes((w.n_out + rc::kSincMfmaTile - 1) / rc::kSincMfmaTile);
    return b;
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

rc_status rc_server_create(rc_context ctx, const rc_sinc *k, int64_t mem_budget_bytes, int32_t max_batch,
                           rc_server *out)
{
    if (!ctx || !out)
        return RC_ERR_INVALID_ARG;
    *out = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->last_error.clear();
        rc_status st = check_sinc(ctx, k);
        if (st != RC_OK)
            return st;
        if (mem_budget_bytes <= 0 || max_batch <= 0)
            return fail(ctx, RC_ERR_INVALID_ARG, "mem_budget_bytes and max_batch must be > 0");
    }
    rc_server srv = new (std::nothrow) rc_server_s();
    if (!srv)
        return RC_ERR_OUT_OF_MEMORY;
    srv->ctx = ctx;
    srv->k = *k;
    srv->budget = mem_budget_bytes;
    srv->max_batch = max_batch;
    {
        DeviceGuard g(ctx->device);
        if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
            delete srv;
            return RC_ERR_DEVICE;
        }
    }
    try {
        srv->launcher = std::thread(server_launcher, srv);
        srv->completer = std::thread(server_completer, srv);
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv_queue.notify_all();
        if (srv->launcher.joinable())
            srv->launcher.join();
        if (srv->completer.joinable())
            srv->completer.join();
        (void)hipStreamDestroy(srv->stream);
        delete srv;
        return RC_ERR_OUT_OF_MEMORY;
    }
    *out = srv;
    return RC_OK;
}

rc_status rc_server_submit(rc_server srv, const rc_request *req, int64_t *ticket)
{
    if (!srv || !req || !ticket)
        return RC_ERR_INVALID_ARG;
    *ticket = 0;
    const PulseWork w{reinterpret_cast<const float2 *>(req->x), reinterpret_cast<float2 *>(req->y), req->n_in,
                      req->n_out, req->fs_hz, req->alpha, req->tec_el_per_m2, req->carrier_hz, req->flags,
                      req->direction};
    {
        std::lock_guard<std::mutex> lk(srv->ctx->mu);
        srv->ctx->last_error.clear();
        if (!req->x || !req->y)
            return fail(srv->ctx, RC_ERR_INVALID_ARG, "NULL sample pointer");
        rc_status st = validate_pulse(srv->ctx, w, "request: ");
        if (st != RC_OK)
            return st;
        if ((w.flags & RC_DO_DOPPLER) && overlaps(req->x, w.n_in * 8, req->y, w.n_out * 8))
            return fail(srv->ctx, RC_ERR_INVALID_ARG, "request: x and y overlap");
        if (!(w.flags & RC_DO_DOPPLER) && req->x != req->y && overlaps(req->x, w.n_in * 8, req->y, w.n_out * 8))
            return fail(srv->ctx, RC_ERR_INVALID_ARG, "request: x and y partially overlap");
    }
    const int64_t bytes = request_bytes(srv->ctx, w, srv->k);
    // the request reads x only after the work enqueued on req->stream so far
    hipEvent_t ready = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->ready_pool.empty()) {
            ready = srv->ready_pool.back();
            srv->ready_pool.pop_back();
        }
    }
    {
        DeviceGuard g(srv->ctx->device);
        hipError_t e = ready ? hipSuccess : hipEventCreateWithFlags(&ready, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(ready, static_cast<hipStream_t>(req->stream));
        if (e != hipSuccess) {
            if (ready) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->ready_pool.push_back(ready);
            }
            std::lock_guard<std::mutex> lk(srv->ctx->mu);
            return device_fail(srv->ctx, e, "request: recording its stream");
        }
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto give_back = [&] { srv->ready_pool.push_back(ready); };
    if (srv->stop) {
        give_back();
        return RC_ERR_INVALID_ARG;
    }
    if (bytes > srv->budget) {
        srv->rejected += 1;
        give_back();
        return RC_ERR_UNSUPPORTED;  // can never be admitted under this budget
    }
    if (srv->in_flight_bytes + bytes > srv->budget) {
        srv->rejected += 1;
        give_back();
        return RC_ERR_BUSY;
    }
    const auto now = rc_server_s::clock::now();
    if (!srv->have_first) {
        srv->have_first = true;
        srv->first_submit = now;
    }
    const int64_t t = srv->next_ticket++;
    srv->in_flight_bytes += bytes;
    srv->submitted += 1;
    srv->tickets.emplace(t, rc_server_s::Ticket{});
    srv->queue.push_back({t, w, bytes, now, ready});
    srv->cv_queue.notify_one();
    *ticket = t;
    return RC_OK;
}

int64_t rc_server_request_bytes(rc_server srv, const rc_request *req)
{
    if (!srv || !req)
        return -1;
    const PulseWork w{reinterpret_cast<const float2 *>(req->x), reinterpret_cast<float2 *>(req->y), req->n_in,
                      req->n_out, req->fs_hz, req->alpha, req->tec_el_per_m2, req->carrier_hz, req->flags,
                      req->direction};
    std::lock_guard<std::mutex> lk(srv->ctx->mu);
    return request_bytes(srv->ctx, w, srv->k);
}

rc_status rc_server_poll(rc_server srv, int64_t ticket, int32_t *done)
{
    if (!srv || !done)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end())
        return RC_ERR_INVALID_ARG;
    *done = it->second.done ? 1 : 0;
    if (it->second.done) {
        const rc_status st = it->second.status;
        srv->tickets.erase(it);
        return st;
    }
    return RC_OK;
}

rc_status rc_server_wait(rc_server srv, int64_t ticket)
{
    if (!srv)
        return RC_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (ticket == 0) {  // everything submitted so far
        const int64_t target = srv->submitted;
        srv->cv_done.wait(lk, [&] { return srv->completed >= target; });
        rc_status st = RC_OK;
        for (auto it = srv->tickets.begin(); it != srv->tickets.end();) {
            if (it->second.done) {
                if (it->second.status != RC_OK)
                    st = it->second.status;
                it = srv->tickets.erase(it);
            } else {
                ++it;
            }
        }
        return st;
    }
    if (srv->tickets.find(ticket) == srv->tickets.end())
        return RC_ERR_INVALID_ARG;
    // another thread's wait-for-all may consume the ticket once it is done
    srv->cv_done.wait(lk, [&] {
        auto f = srv->tickets.find(ticket);
        return f == srv->tickets.end() || f->second.done;
    });
    auto f = srv->tickets.find(ticket);
    if (f == srv->tickets.end())
        return RC_OK;
    const rc_status st = f->second.status;
    srv->tickets.erase(f);
    return st;
}

rc_status rc_server_stats(rc_server srv, rc_server_stats_t *out)
{
    if (!srv || !out)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    rc_server_stats_t s{};
    s.submitted = srv->submitted;
    s.completed = srv->completed;
    s.rejected = srv->rejected;
    s.batches = srv->batches;
    s.mean_batch = srv->batches ? (double)srv->batched_reqs / (double)srv->batches : 0.0;
    s.latency_ms_p50 = percentile(srv->latency_ms, 0.50);
    s.latency_ms_p99 = percentile(srv->latency_ms, 0.99);
    s.latency_ms_max = srv->latency_ms.empty() ? 0.0 : *std::max_element(srv->latency_ms.begin(), srv->latency_ms.end());
    const double span = srv->have_first && srv->completed
                            ? std::chrono::duration<double>(srv->last_done - srv->first_submit).count()
                            : 0.0;
    s.samples_per_s = span > 0.0 ? (double)srv->samples / span : 0.0;
    *out = s;
    return RC_OK;
}

rc_status rc_server_reset_stats(rc_server srv)
{
    if (!srv)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted -= srv->completed;
    srv->completed = srv->rejected = srv->batches = srv->batched_reqs = srv->samples = 0;
    srv->latency_ms.clear();
    srv->have_first = false;
    return RC_OK;
}

rc_status rc_server_destroy(rc_server srv)
{
    if (!srv)
        return RC_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_queue.notify_all();
    srv->launcher.join();  // launches what is queued, then stops
    srv->completer.join(); // waits for every launched batch
    {
        DeviceGuard g(srv->ctx->device);
        for (hipEvent_t e : srv->event_pool)
            (void)hipEventDestroy(e);
        for (hipEvent_t e : srv->ready_pool)
            (void)hipEventDestroy(e);
        (void)hipStreamDestroy(srv->stream);
    }
    delete srv;
    return RC_OK;
}

rc_status rc_set_sinc_engine(rc_context ctx, int32_t engine)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (engine != RC_SINC_AUTO && engine != RC_SINC_VALU && engine != RC_SINC_DIRECT)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown sinc engine");
    ctx->sinc_engine = engine;
    return RC_OK;
}

rc_status rc_set_bank_engine(rc_context ctx, int32_t engine)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (engine != RC_BANK_ENGINE_AUTO && engine != RC_BANK_ENGINE_FARROW && engine != RC_BANK_ENGINE_PER_HYPOTHESIS)
        return fail(ctx, RC_ERR_INVALID_ARG, "unknown bank engine");
    ctx->bank_engine = engine;
    return RC_OK;
}

rc_status rc_set_fft_levels(rc_context ctx, int64_t n, const int32_t *levels, int32_t count)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (count < 0 || (count > 0 && !levels))
        return fail(ctx, RC_ERR_INVALID_ARG, "NULL levels or negative count");
    if (count == 0) {
        ctx->fft_levels.erase(n);
    } else {
        std::vector<int> lv(levels, levels + count);
        FftPlan probe;
        if (rc::build_fft_plan_levels(n, lv, probe) != hipSuccess)
            return fail(ctx, RC_ERR_INVALID_ARG,
                        "levels must be powers of two in [2, 256], at most 3, with 4096 times their product = n");
        ctx->fft_levels[n] = lv;
    }
    ctx->plans.erase(n);  // rebuilt with the new split on its next use
    return RC_OK;
}

rc_status rc_set_sinc_grid(rc_context ctx, int32_t half_width, int32_t wg_per_cu)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if ((half_width != 64 && half_width != 128) || wg_per_cu < 0 || wg_per_cu > 64)
        return fail(ctx, RC_ERR_INVALID_ARG, "half_width must be 64 or 128 and wg_per_cu in [0, 64]");
    ctx->sinc_wg_per_cu[half_width == 128 ? 1 : 0] = wg_per_cu;
    return RC_OK;
}

rc_status rc_set_bluestein_chunk(rc_context ctx, int64_t bytes)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->last_error.clear();
    if (bytes < 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "bytes must be >= 0");
    ctx->bluestein_chunk = bytes;
    return RC_OK;
}

rc_status rc_load_tuning(rc_context ctx, const char *path)
{
    if (!ctx || !path)
        return RC_ERR_INVALID_ARG;
    std::string text, err;
    {
        std::FILE *f = std::fopen(path, "rb");
        if (!f) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            return fail(ctx, RC_ERR_INVALID_ARG, std::string("cannot open the tuning file ") + path);
        }
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof buf, f)) > 0)
            text.append(buf, got);
        std::fclose(f);
    }
    Json root;
    if (!parse_json(text, root, err) || root.kind != Json::Object) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        return fail(ctx, RC_ERR_INVALID_ARG, std::string("tuning file ") + path + ": " + (err.empty() ? "not an object" : err));
    }
    auto bad = [&](const std::string &why) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        return fail(ctx, RC_ERR_INVALID_ARG, std::string("tuning file ") + path + ": " + why);
    };
    // validate everything first, then apply
    std::vector<std::pair<int64_t, std::vector<int32_t>>> lv;
    std::vector<std::pair<int32_t, int32_t>> grid;
    int64_t chunk = -1;
    for (const auto &kv : root.obj) {
        if (kv.first == "fft_levels") {
            if (kv.second.kind != Json::Object)
                return bad("fft_levels must be an object");
            for (const auto &e : kv.second.obj) {
                if (e.second.kind != Json::Array)
                    return bad("fft_levels entries must be arrays");
                std::vector<int32_t> v;
                for (const auto &q : e.second.arr) {
                    if (q.kind != Json::Number)
                        return bad("fft_levels values must be numbers");
                    v.push_back((int32_t)q.num);
                }
                char *end = nullptr;
                const long long n = std::strtoll(e.first.c_str(), &end, 10);
                if (!end || *end)
                    return bad("fft_levels keys must be transform lengths");
                lv.emplace_back((int64_t)n, v);
            }
        } else if (kv.first == "sinc_grid") {
            if (kv.second.kind != Json::Object)
                return bad("sinc_grid must be an object");
            for (const auto &e : kv.second.obj) {
                if (e.second.kind != Json::Number)
                    return bad("sinc_grid values must be numbers");
                grid.emplace_back((int32_t)std::atoi(e.first.c_str()), (int32_t)e.second.num);
            }
        } else if (kv.first == "bluestein_chunk_bytes") {
            if (kv.second.kind != Json::Number)
                return bad("bluestein_chunk_bytes must be a number");
            chunk = (int64_t)kv.second.num;
        }  // other keys (the measurements behind the choices) are ignored
    }
    for (const auto &e : lv) {
        const rc_status st = rc_set_fft_levels(ctx, e.first, e.second.data(), (int32_t)e.second.size());
        if (st != RC_OK)
            return st;
    }
    for (const auto &e : grid) {
        const rc_status st = rc_set_sinc_grid(ctx, e.first, e.second);
        if (st != RC_OK)
            return st;
    }
    if (chunk >= 0)
        return rc_set_bluestein_chunk(ctx, chunk);
    return RC_OK;
}

rc_status rc_set_mem_budget(rc_context ctx, int64_t bytes)
{
    if (!ctx)
        return RC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (bytes < 0)
        return fail(ctx, RC_ERR_INVALID_ARG, "the memory budget must be >= 0");
    ctx->mem_budget = bytes;
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
                                            "k_mf_tile_list", "k_bluestein", "k_farrow_z", "k_farrow_bank",
                                            "k_paper_sinc", "k_linear", "k_tone", "k_pq"};

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
