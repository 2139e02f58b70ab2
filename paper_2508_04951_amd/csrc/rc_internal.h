// rc_internal.h -- types shared by the HIP sources of librc.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rc.h"

namespace rc {

// Optional kernel timing: while `on`, each launch is bracketed by two HIP events on its stream.
enum KernelGroup {
    kKSincFast = 0,
    kKSincDirect,
    kKFftStridedFwd,
    kKFftRowsIono,
    kKFftStridedInv,
    kKSincMfma,
    kKSincTiles,
    kKBluestein,
    kKFarrowZ,
    kKFarrowBank,
    kKPaperSinc,
    kKLinear,
    kKTone,
    kKPq,
    kKGroups
};
extern const char *const kKernelNames[kKGroups];

struct Profiler {
    bool on = false;
    struct Span {
        int group;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    double total_ms[kKGroups] = {0};
    int64_t launches[kKGroups] = {0};
    int open_group = -1;
    hipEvent_t open_a = nullptr;
    hipEvent_t take();
    void begin(int group, hipStream_t s);
    void end(hipStream_t s);
    hipError_t collect();  // wait for recorded spans and accumulate them
    void release();
};

// Speed of light, exact (SI).  e, m_e and eps0 (CODATA 2022) enter only K2 / E, evaluated on
// the host in long double next to the dispersive phase.
constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------------------
// Doppler resampling
// ---------------------------------------------------------------------------------------

// Kaiser taper as a power series in s = 1 - x^2:  K(x) = sum_j c[j] s^j,  |x| < 1.
// From I0(z) = sum_j (z^2/4)^j / (j!)^2 with z^2 = beta^2 s, divided by I0(beta).
// All terms are positive for s in [0, 1], so the Horner sum has no cancellation.
struct KaiserPoly {
    int n;          // number of terms
    double c[56];   // c[j] = (beta^2/4)^j / (j!)^2 / I0(beta)
    int nf;         // terms a float32 evaluation needs: the rest sum to below 2^-27 of K(0) = 1
    float cf[56];   // c[j] rounded to float32
};

// Global-memory view of a device pointer.  Kernels read their pointers from job descriptors,
// so the compiler cannot tell them from LDS and emits flat accesses, which also count against
// the LDS wait counter: every wait for an LDS result would then wait for outstanding HBM loads
// too.  Accesses through this view compile to global_* instructions.
#ifdef __HIP_DEVICE_COMPILE__
#define RC_GLOBAL_AS __attribute__((address_space(1)))
#else
#define RC_GLOBAL_AS  // the host pass has no device address spaces
#endif
template <class T>
__device__ __forceinline__ RC_GLOBAL_AS T *gmem(T *p)
{
    return (RC_GLOBAL_AS T *)p;
}

template <class T>
__device__ __forceinline__ T gload(const T *p, int64_t i)
{
    return gmem(p)[i];
}

// Streaming store of one complex sample (non-temporal hint): large outputs read by the next
// kernel on other XCDs gain nothing from staying in this XCD's L2.
__device__ __forceinline__ void store_nt(float2 *p, float2 v)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(f2v{v.x, v.y}, (RC_GLOBAL_AS f2v *)p);
}

// One resampling job (one pulse).  Pointers are device addresses.
struct SincJob {
    const float2 *x;
    float2 *y;
    int64_t n_in;
    int64_t n_out;
    double alpha;
    int64_t tile0;  // matrix-core path: index of this job's first tile in the batch's tile list
};

// Tile geometry of the windowed fast path: each wave owns 256 consecutive outputs
// (4 per lane); a 256-thread workgroup owns 1024.
constexpr int kSincLanesOut = 4;
constexpr int kSincWaveOut = 64 * kSincLanesOut;
constexpr int kSincWgOut = 4 * kSincWaveOut;
// |alpha - 1| bound of the fast path: keeps the per-tile sample-position drift
// |alpha-1| * 127.5 below 0.013 samples, where the quadratic-in-drift weights are
// accurate to ~1e-7 per tap.
constexpr double kSincFastMaxEps = 1.0e-4;

bool sinc_fast_eligible(double alpha, const rc_sinc &k);

// Matrix-core path (Kaiser, H = 64 or 128): a 2048-output tile takes its tap weights from a
// quartic in the drift tabulated on a grid of 129 phases, so |alpha - 1| * 1023.5 must stay
// below ~0.061 samples.
constexpr double kSincMfmaMaxEps = 6.0e-5;
constexpr int kSincMfmaTile = 2048;
struct MfmaSincConst {
    double node[5];   // Chebyshev nodes of [-1, 1]
    double vinv[25];  // inverse Vandermonde matrix: a_r = sum_i vinv[5 r + i] h(node_i)
};
bool sinc_mfma_eligible(double alpha, const rc_sinc &k);
// Device table of the B fragments for every grid phase (built once per (H, beta)).
hipError_t build_sinc_mfma_table(int half_width, double beta, void **dev, std::vector<void *> &allocs);
// Batches of more tiles than the resident workgroups run persistent workgroups over a tile list
// sorted by phase; the list needs `sinc_mfma_work_bytes(ntiles)` of device workspace.
bool sinc_mfma_uses_list(int half_width, int64_t ntiles, int wg_per_cu = 0);
size_t sinc_mfma_work_bytes(int64_t ntiles);
// Where the tile-list kernels may run: on `stream` once `after` (the descriptor upload) has
// completed, signalling `done`, which the compute stream waits for before the resampling kernel.
// They read only the call's descriptors and write only its workspace, so on a side stream they
// overlap whatever earlier work the compute stream still has queued.
struct TileStream {
    hipStream_t stream;
    hipEvent_t after;  // may be null
    hipEvent_t done;
};
// What launch_sinc_mfma enqueues when it uses a tile list: the list and then the resampling
// kernel; the list alone (it depends only on the job descriptors); or the resampling kernel over
// a list built earlier in the same workspace (a captured graph replaying a fixed batch).
enum class TileListMode { BuildAndRun, BuildOnly, RunOnly };
// jobs_dev (device array, tile0 set) or job_inline (one job, tile0 = 0); `work` is the workspace
// when sinc_mfma_uses_list(), else unused.  With ts null the tile list is built on s.
hipError_t launch_sinc_mfma(const SincJob *jobs_dev, const SincJob *job_inline, int njobs,
                            int64_t max_out, int64_t ntiles, void *work, int half_width,
                            const void *table, hipStream_t s, Profiler *prof, const TileStream *ts = nullptr,
                            TileListMode mode = TileListMode::BuildAndRun, int wg_per_cu = 0);
KaiserPoly make_kaiser_poly(double beta);
size_t sinc_fast_lds_bytes(int half_width);

// Launchers (return the hipError_t of the launch).
hipError_t launch_sinc_fast(const SincJob *jobs_dev, const SincJob *job_inline, int njobs,
                            int64_t max_out, int half_width, const KaiserPoly &kp,
                            hipStream_t s, Profiler *prof);
hipError_t launch_sinc_direct(const SincJob *jobs_dev, const SincJob *job_inline, int njobs,
                              int64_t max_out, const rc_sinc &k, const KaiserPoly &kp,
                              int64_t max_taps, hipStream_t s, Profiler *prof);

// ---------------------------------------------------------------------------------------
// Doppler bank (Farrow filter bank, bank.hip)

constexpr int kFarrowOrders = 8;            // Chebyshev terms per tap weight
constexpr int kFarrowMaxHalfWidth = 256;
constexpr double kFarrowMaxAlpha = 2.0;     // keeps a workgroup's Z rows within LDS
struct FarrowPlan {
    int n_hyp = 0;
    std::vector<double> alpha;              // sorted ascending
    std::vector<int> hyp;                   // original hypothesis index of each sorted entry
    struct Group {
        int first, count;
    };
    std::vector<Group> groups;              // consecutive sorted hypotheses sharing a workgroup
    int max_rows = 0;                       // Z rows one workgroup stages
    int64_t F = 0;                          // Z rows computed (input positions 0 .. F-1)
    size_t z_bytes = 0;
    size_t lds_bytes = 0;
};
bool farrow_eligible(const rc_sinc &k, const double *alphas, int n_hyp);
hipError_t build_farrow_coef(const rc_sinc &k, void **dev, std::vector<void *> &allocs);
FarrowPlan plan_farrow_bank(int64_t n, int64_t n_out, int H, const double *alphas, int n_hyp);
size_t farrow_desc_bytes(const FarrowPlan &p);
void farrow_pack_desc(const FarrowPlan &p, char *host);
// desc_dev: farrow_pack_desc() uploaded; z_work: p.z_bytes of device memory
// precision: RC_BANK_FP16X3 | RC_BANK_BF16X3 | RC_BANK_FP32 (the Z filter's contraction)
hipError_t launch_farrow_bank(const FarrowPlan &p, const float2 *x, int64_t n, float2 *y, int64_t n_out, int H,
                              int precision, const float *coef, const void *desc_dev, void *z_work, hipStream_t s,
                              Profiler *prof);

// ---------------------------------------------------------------------------------------
// FFT / ionosphere
// ---------------------------------------------------------------------------------------

// Every FFT pass works on a tile of 4096 complex samples (32 KiB of LDS) with 256 threads.
constexpr int kFftTile = 4096;
constexpr int kFftThreads = 256;
constexpr int kFftMaxLevels = 4;

// Numerator of the dispersive phase of Eq (15)/(16) in quarter turns: bin frequency f turns
// by (hi + lo) / f quarter turns, hi + lo = s * 8 K2 / c (= s * 4 pi K2 / c over pi / 2), s = -1
// for correction (Eq 16) and +1 for distortion (Eq 15), evaluated on the host in long double.
// xprec asks for the quotient in double-double arithmetic: set when some bin's phase exceeds
// 2^26 quarter turns (a carrier within about fs / 2 of 0 Hz), where a float64 quotient would be
// uncertain by more than 1e-7 quarter turn.  hi == 0 means no phase.
struct PhaseNum {
    double hi, lo;
    int xprec;
};

// Per-pulse ionospheric parameters; f_k = carrier + fs * kk / n.
struct IonoJob {
    const float2 *x;  // input of the first pass (may equal y)
    float2 *y;        // output; every later pass runs in place on y
    PhaseNum phase;
    double carrier;
    double fs;
    // When set, the spectrum is also multiplied by this table (in the transform's native bin
    // order, see launch_fft_forward), conjugated if conj_mult: a circular convolution or, with
    // the conjugate, a correlation.  The dispersive phase applies on top unless phase.hi is 0.
    const float2 *mult;
    int conj_mult;
};

// Decomposition of an n-point transform into levels L_0 x L_1 x ... x L_{d-1}
// (row-major, L_{d-1} contiguous).  Strided levels are <= 256 long, the last <= 4096.
struct FftPlan {
    int64_t n = 0;
    int levels = 0;
    int len[kFftMaxLevels] = {0, 0, 0, 0};
    int log2len[kFftMaxLevels] = {0, 0, 0, 0};
};

hipError_t build_fft_plan(int64_t n, FftPlan &plan, std::vector<void *> &allocs);
// The plan of a power-of-two n > 4096 with the given strided levels (each a power of two in
// [2, 256], at most kFftMaxLevels - 1 of them) before the 4096-point contiguous level; their
// product times 4096 must be n.  hipErrorInvalidValue otherwise.
hipError_t build_fft_plan_levels(int64_t n, const std::vector<int> &strided, FftPlan &plan);
hipError_t make_base_twiddles(float2 **dev);  // exp(-2 pi i q / 4096), q < 4096

// What the contiguous FFT pass multiplies each bin by: the dispersive phase (the ionospheric
// operator) or, for a job with a `mult` table, the table alone (a convolution); or the table,
// conjugated if the job says so, times the phase (a correlation with the correction).  Every job
// of one launch takes the same kind.
enum RowFactor { kRowPhaseOrTable = 0, kRowTablePhase = 1 };
// Full ionospheric operator for njobs pulses of the same length plan.n: forward FFT, the
// per-bin factor, inverse FFT with 1/n.
hipError_t launch_iono(const FftPlan &plan, const float2 *tw4096, const IonoJob *jobs_dev,
                       const IonoJob *job_inline, int njobs, hipStream_t s, Profiler *prof,
                       int factor = kRowPhaseOrTable);
// Forward FFT only, the spectrum left in the native bin order of the multi-level transform:
// bin k sits at (row r) * L + l where L is the last level and row r holds bins
// kout(r) + (n / L) l (kout = the digit-reversed row index).  For a one-level plan the order
// is natural.  Used to build `mult` tables.
hipError_t launch_fft_forward(const FftPlan &plan, const float2 *tw4096, const IonoJob *jobs_dev,
                              const IonoJob *job_inline, int njobs, hipStream_t s, Profiler *prof);

// dst[i] = r[i] for i < n_rep, 0 up to n (a replica zero-padded to a transform length).
hipError_t launch_pad(const float2 *r, int64_t n_rep, float2 *dst, int64_t n, hipStream_t s);

// Ionospheric operator of a length n that is not a power of two (Bluestein): the N-point DFT
// as a chirp convolution of power-of-two length m >= 2n - 1 (bluestein_m).  Each pulse needs
// 2 m complex values of workspace: the convolution buffer a and the chirp spectrum b = a + m.
struct BluesteinJob {
    const float2 *x;  // input, n samples
    float2 *y;        // output, n samples (may equal x)
    float2 *a;        // workspace: a[0, m) and b = a + m
    int64_t n;
    PhaseNum phase;                 // as in IonoJob
    double carrier, fs;
    // When set, the spectrum is also multiplied by conj(corr[k]) (natural bin order, n values):
    // the cross-correlation with the signal whose spectrum corr holds (pulse compression).
    const float2 *corr;
};
int64_t bluestein_m(int64_t n);
size_t bluestein_work_bytes(int64_t n);  // 2 m complex values
// njobs pulses whose lengths share m = mplan.n, in one launch sequence.  With jobs_dev null,
// the single job `inl` runs (njobs must be 1; no device descriptors needed).  Otherwise
// jobs_dev holds the njobs BluesteinJob and ffts_dev 2 njobs IonoJob: the chirp transforms
// {b_j, b_j} and then the convolutions {a_j, a_j, mult = b_j}.  max_n bounds every job's n.
hipError_t launch_iono_bluestein(const FftPlan &mplan, const float2 *tw4096, const BluesteinJob *jobs_dev,
                                 const IonoJob *ffts_dev, const BluesteinJob &inl, int njobs, int64_t max_n,
                                 hipStream_t s, Profiler *prof);
// The forward DFT alone of one job by Bluestein's chirp convolution: y[k] = DFT_n(x)[k] in natural
// bin order, unnormalised (phase and corr unused).  y may equal x.
hipError_t launch_bluestein_forward(const FftPlan &mplan, const float2 *tw4096, const BluesteinJob &inl,
                                    hipStream_t s, Profiler *prof);

// ---------------------------------------------------------------------------------------
// The paper's other resampling methods (methods.hip)
// ---------------------------------------------------------------------------------------

// One call of the paper's sinc kernels (App. C): 2h + 1 taps centred on the nearest input.
struct PaperArgs {
    const float2 *x;
    float2 *y;
    int64_t n_in, n_out;
    double alpha;
    int64_t h;
    int lut_size;        // Alg. 2 table entries
    double dx, inv_dx;   // Alg. 2 table spacing (h + 1/2) / (lut_size - 1) and its inverse
};
// Dynamic LDS of the tiled kernel (Alg. 3): the inputs of 256 consecutive outputs.
size_t paper_tiled_lds_bytes(double alpha, int h);
// variant: RC_PAPER_DIRECT / RC_PAPER_TILED / RC_PAPER_LUT; blocks 0: one output per thread.
hipError_t launch_paper_sinc(const PaperArgs &a, int variant, int blocks, hipStream_t s, Profiler *prof);
hipError_t launch_linear(const float2 *x, int64_t n_in, float2 *y, int64_t n_out, double alpha, hipStream_t s,
                         Profiler *prof);
// y[m] = x[m] exp(2 pi i nu m), nu in cycles per sample; y may equal x.
hipError_t launch_tone(const float2 *x, float2 *y, int64_t n, double nu, hipStream_t s, Profiler *prof);
// FFT P/Q resampling of x (n_in samples) to ni samples, written to y[0, n_out) (zeros past ni),
// optionally turned by exp(2 pi i nu m).  Workspace: X (n_in complex), Y (ni complex) and `work`
// (bluestein_work_bytes of the larger length).  ni == n_in: no transform, y is x (turned).
struct PqArgs {
    const float2 *x;
    float2 *y;
    int64_t n_in, ni, n_out;
    float2 *X, *Y, *work;
    int tone;
    double nu;
};
hipError_t launch_pq(const PqArgs &a, const FftPlan &plan_in, const FftPlan &plan_out, const float2 *tw4096,
                     hipStream_t s, Profiler *prof);

}  // namespace rc

// The context behind the opaque rc_context handle.
struct rc_context_s {
    int device = 0;
    std::mutex mu;
    std::string last_error;
    float2 *tw4096 = nullptr;                  // base twiddles exp(-2 pi i q / 4096)
    std::map<int64_t, rc::FftPlan> plans;      // by transform length
    std::map<std::pair<int, double>, void *> mfma_tables;  // by (half width, Kaiser beta)
    std::map<std::pair<std::pair<int, int>, double>, void *> farrow_coefs;  // by ((H, window), beta)
    std::vector<void *> allocs;                // every device allocation owned
    // descriptor staging: a ring of pinned host + device slots; a slot is reused only after the
    // work that read it has completed (its event)
    struct DescSlot {
        void *host = nullptr;
        void *dev = nullptr;
        size_t host_cap = 0;
        size_t dev_cap = 0;
        hipEvent_t done = nullptr;
        hipEvent_t uploaded = nullptr;  // the upload of this slot's descriptors (copy stream)
        bool pending = false;
    };
    // descriptors go up on their own stream, so a batch's upload overlaps the previous batch's
    // kernels; the compute stream waits for it by event
    hipStream_t copy_stream = nullptr;
    // the matrix-core tile list of a call is built on its own stream (see rc::TileStream)
    hipStream_t tile_stream = nullptr;
    hipEvent_t tiles_done = nullptr;
    static constexpr int kDescSlots = 4;
    DescSlot desc[kDescSlots];
    int desc_next = 0;
    rc::Profiler prof;
    int sinc_engine = 0;  // RC_SINC_AUTO / RC_SINC_VALU / RC_SINC_DIRECT
    int bank_engine = 0;  // RC_BANK_ENGINE_AUTO / _FARROW / _PER_HYPOTHESIS
    int64_t mem_budget = 0;  // cap on the slots' device workspace in bytes (rc_set_mem_budget); 0: none
    // tuning (rc_set_fft_levels, rc_set_sinc_grid, rc_set_bluestein_chunk, rc_load_tuning)
    std::map<int64_t, std::vector<int>> fft_levels;  // strided levels by transform length
    int sinc_wg_per_cu[2] = {0, 0};                   // matrix-core grid at H = 64, 128 (0: occupancy)
    int64_t bluestein_chunk = 0;                      // Bluestein chunk workspace cap (0: default)
    // device address of this device's copy of the library's static workspace (the
    // no-allocation entry point's Bluestein buffers), looked up once per device at rc_create
    float2 *static_scratch = nullptr;
};
