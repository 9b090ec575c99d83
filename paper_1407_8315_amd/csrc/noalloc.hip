// sft_exact_noalloc: exactly K-sparse recovery of one signal (the path of
// sft_exact) for callers that cannot allocate device memory.  The workspace a
// plan would hipMalloc (syndromes, queues, staging, ranking scratch, tables,
// the signal's descriptor and work items) lives in one file-scope device
// array, `scratch`, of fixed size; each GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to the
// device: at the first call on a device it takes the array's address on that
// device with hipGetSymbolAddress and keeps it per device.
//
// A call enqueues, on the caller's stream and in order: (first call on a
// device, or a call under stream capture) a kernel that fills the twiddle and
// unit-root tables; a set-up kernel that copies the signal's descriptor, work
// items and output pointers (passed by value) into the array; then the same
// kernels sft_exact runs, with the stage's parallel branches in series.  No
// hipMalloc, hipFree, memset or copy is issued, so the call can be captured
// into a HIP graph.  Every call on a GPU shares that GPU's array: calls must be
// ordered by the caller (one stream, or synchronisation between streams);
// overlapping calls race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"
#include "plan_host.h"
#include "sft.h"

namespace sft {
namespace {

// Limits of the static workspace: one-pass FFTs only (M up to 8192 points
// with FP32 FFTs, 4096 with FP64 FFTs), L up to 4 (2L = 8 lines), d = N/M up
// to 2^16 (the unit-root table).
constexpr int kNaTw32Log2 = 13;
constexpr int kNaTw64Log2 = 12;
constexpr int kNaOmLog2 = 16;
constexpr int64_t kNaMaxM32 = int64_t(1) << kNaTw32Log2;
constexpr int64_t kNaMaxM64 = int64_t(1) << kNaTw64Log2;
constexpr int64_t kNaMaxD = int64_t(1) << kNaOmLog2;
constexpr int kNaLines = 2 * kMaxL;
constexpr int64_t kNaMaxBins = kNaMaxM32;                       // list capacity (bins of the signal)
constexpr int64_t kNaMaxStage = kNaMaxBins * kMaxL;            // staging entries, M * L
constexpr int kNaMaxBinItems = (int)(kNaMaxBins / kBlock);
constexpr int kNaMaxActItems = (int)((kNaMaxBins + kActivityTile - 1) / kActivityTile);
static_assert(kNaMaxM32 == kFftPointsF32 && kNaMaxM64 == kFftPointsF64, "one-pass FFT limits");

constexpr int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

int ilog2_na(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// Per-call description, passed by value to the set-up kernel.
struct NaArgs {
    SigDev sig;
    IoDev io;
    int64_t shifts[kNaLines];
    int4 synd_items[kNaLines];
    int4 pair_items[kMaxL];
    int2 bin_items[kNaMaxBinItems];
    int2 act_items[kNaMaxActItems];
};
static_assert(sizeof(NaArgs) <= 2048, "kernel argument block");

// Byte offsets of the regions of the array.
constexpr int64_t kOffArgs = 0;
constexpr int64_t kOffTw32 = align256(kOffArgs + (int64_t)sizeof(NaArgs));
constexpr int64_t kOffTw64 = align256(kOffTw32 + (int64_t)sizeof(float2) * kNaMaxM32);
constexpr int64_t kOffOmega = align256(kOffTw64 + (int64_t)sizeof(double2) * kNaMaxM64);
constexpr int64_t kOffSynd = align256(kOffOmega + (int64_t)sizeof(double2) * kNaMaxD);
constexpr int64_t kSyndBytes = std::max<int64_t>(kNaLines * kNaMaxM32 * (int64_t)sizeof(float2),
                                                 kNaLines * kNaMaxM64 * (int64_t)sizeof(double2));
constexpr int64_t kOffEpart = align256(kOffSynd + kSyndBytes);
constexpr int64_t kOffSigma = align256(kOffEpart + (int64_t)sizeof(double) * kNaLines);
constexpr int64_t kOffEbin = align256(kOffSigma + (int64_t)sizeof(double));
constexpr int64_t kOffSel = align256(kOffEbin + (int64_t)sizeof(double));
constexpr int64_t kOffCnt = align256(kOffSel + (int64_t)sizeof(SelDev));
constexpr int64_t kOffWork = align256(kOffCnt + (int64_t)sizeof(SigCounters));
constexpr int64_t kOffStLoc = align256(kOffWork + (int64_t)sizeof(WorkCounters));
constexpr int64_t kOffStVal = align256(kOffStLoc + (int64_t)sizeof(int64_t) * kNaMaxStage);
constexpr int64_t kOffKidx = align256(kOffStVal + (int64_t)sizeof(double2) * kNaMaxStage);
constexpr int64_t kOffRkA = align256(kOffKidx + (int64_t)sizeof(int) * kNaMaxStage);
constexpr int64_t kOffRkB = align256(kOffRkA + (int64_t)sizeof(double) * kNaMaxStage);
constexpr int64_t kOffRkI = align256(kOffRkB + (int64_t)sizeof(long long) * kNaMaxStage);
constexpr int64_t kOffRkR = align256(kOffRkI + (int64_t)sizeof(int) * kNaMaxStage);
constexpr int64_t kOffActive = align256(kOffRkR + (int64_t)sizeof(int) * kNaMaxStage);
constexpr int64_t kOffQlist = align256(kOffActive + (int64_t)sizeof(int2) * kNaMaxBins);
constexpr int64_t kScratchBytes = align256(kOffQlist + (int64_t)sizeof(int2) * kNaMaxBins * kQueues);
static_assert(kScratchBytes <= (int64_t(6) << 20), "the static workspace stays under 6 MiB");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// e^{-2 pi i q / 2^log2n} (both precisions) and e^{+2 pi i q / 2^log2n}, the
// tables a plan builds on the host, here on the device (FP64 cos and sin of
// the same argument).
__global__ void na_tables_kernel(float2* tw32, double2* tw64, double2* om) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNaMaxM32) {
        const double a = -2.0 * M_PI * (double)i / (double)kNaMaxM32;
        tw32[i] = float2{(float)cos(a), (float)sin(a)};
    }
    if (i < kNaMaxM64) {
        const double a = -2.0 * M_PI * (double)i / (double)kNaMaxM64;
        tw64[i] = double2{cos(a), sin(a)};
    }
    if (i < kNaMaxD) {
        const double a = 2.0 * M_PI * (double)i / (double)kNaMaxD;
        om[i] = double2{cos(a), sin(a)};
    }
}

__global__ void na_setup_kernel(NaArgs a, NaArgs* dst) {
    if (threadIdx.x == 0) *dst = a;
}

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_base[kNaMaxDevices];   // device address of `scratch`, per device
bool g_na_tables[kNaMaxDevices];           // tables written by an eager (not captured) call

#define NA_CHECK(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_error(SFT_E_DEVICE, std::string("sft_exact_noalloc: ") + #call + ": " + hipGetErrorString(e_)); \
    } while (0)

// The array's address on the current device (taken once per device) and the
// tables, enqueued on `stream` unless an earlier eager call wrote them.
sft_status na_prepare(hipStream_t stream, unsigned char** base) {
    int dev = 0;
    NA_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return set_error(SFT_E_UNSUPPORTED, "sft_exact_noalloc: device index above 63");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    NA_CHECK(hipStreamIsCapturing(stream, &cap));
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_base[dev]) {
        void* ptr = nullptr;
        NA_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(SFT_E_DEVICE, "sft_exact_noalloc: no device address for the workspace");
        g_na_base[dev] = (unsigned char*)ptr;
    }
    unsigned char* b = g_na_base[dev];
    if (!g_na_tables[dev]) {
        const int n = (int)std::max(kNaMaxD, kNaMaxM32);
        hipLaunchKernelGGL(na_tables_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                           (float2*)(b + kOffTw32), (double2*)(b + kOffTw64), (double2*)(b + kOffOmega));
        NA_CHECK(hipGetLastError());
        // a captured launch runs only when its graph does: keep writing them
        // until an eager call has
        if (cap == hipStreamCaptureStatusNone) g_na_tables[dev] = true;
    }
    *base = b;
    return SFT_OK;
}

}  // namespace
}  // namespace sft

using namespace sft;

extern "C" sft_status sft_exact_noalloc(const sft_params* params, const void* x_dev, const sft_sparse_out* out,
                                        void* hip_stream) {
    if (!params || !x_dev || !out) return set_error(SFT_E_INVALID, "sft_exact_noalloc: NULL argument");
    if (!out->count_dev || out->capacity < 0 || (out->capacity > 0 && (!out->loc_dev || !out->val_dev)))
        return set_error(SFT_E_INVALID, "sft_exact_noalloc: output list is incomplete");
    if (params->mode != SFT_MODE_EXACT) return set_error(SFT_E_INVALID, "sft_exact_noalloc: mode must be SFT_MODE_EXACT");
    const uint32_t refused = SFT_FLAG_LEARNED | SFT_FLAG_SYNC | SFT_FLAG_CHECK_FINITE | SFT_FLAG_UNKNOWN_K;
    if (params->flags & refused)
        return set_error(SFT_E_UNSUPPORTED,
                         "sft_exact_noalloc: SFT_FLAG_LEARNED, SYNC, CHECK_FINITE and UNKNOWN_K are not available");
    SigHost g;
    std::string msg;
    sft_status s = resolve_params(*params, false, &g, &msg);
    if (s != SFT_OK) return set_error(s, "sft_exact_noalloc: " + msg);
    const bool in64 = g.dtype == SFT_C128;
    const bool fp64 = in64 || (g.flags & SFT_FLAG_FFT64) != 0;
    const int64_t mmax = fp64 ? kNaMaxM64 : kNaMaxM32;
    if (g.m > mmax)
        return set_error(SFT_E_UNSUPPORTED, "sft_exact_noalloc: M = " + std::to_string(g.m) +
                                                " is above the static workspace's limit " + std::to_string(mmax) +
                                                (fp64 ? " (FP64 FFTs)" : " (FP32 FFTs)"));
    if (g.d > kNaMaxD)
        return set_error(SFT_E_UNSUPPORTED, "sft_exact_noalloc: d = N/M = " + std::to_string(g.d) +
                                                " is above the static workspace's limit " + std::to_string(kNaMaxD));

    // descriptor, work items and output pointers of the signal (as a
    // single-signal plan lays them out, every offset 0)
    NaArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sig = sigdev_of(g, kNaMaxD, fp64);
    a.io = IoDev{x_dev, out->loc_dev, (double2*)out->val_dev, out->capacity, out->count_dev};
    for (int l = 0; l < g.S; ++l) a.shifts[l] = l;
    // the 2L consecutive shifts by pair_syndrome_kernel where a plan uses it
    const int pb = (!fp64 && 2 * g.L - 1 < g.d) ? pair_block(g.L, g.m) : 0;
    int n_pair = 0;
    if (pb)
        for (int l0 = 0; l0 < 2 * g.L; l0 += 2 * pb) a.pair_items[n_pair++] = int4{0, l0, 0, 0};
    const int first = pb ? 2 * g.L : 0;
    bool small = false;
    const int nl = fft_lines_per_block(g.m, g.S - first, fp64, &small);
    int n_synd = 0;
    for (int l0 = first; l0 < g.S; l0 += nl) a.synd_items[n_synd++] = int4{0, l0, std::min(nl, g.S - l0), 0};
    int n_bins = 0, n_act = 0;
    for (int64_t b = 0; b < g.m; b += kBlock) a.bin_items[n_bins++] = int2{0, (int)b};
    for (int64_t b = 0; b < g.m; b += kActivityTile) a.act_items[n_act++] = int2{0, (int)b};

    hipStream_t stream = (hipStream_t)hip_stream;
    unsigned char* base = nullptr;
    s = na_prepare(stream, &base);
    if (s != SFT_OK) return s;
    NaArgs* hdr = (NaArgs*)(base + kOffArgs);
    hipLaunchKernelGGL(na_setup_kernel, dim3(1), dim3(64), 0, stream, a, hdr);
    NA_CHECK(hipGetLastError());

    LaunchCtx c{};
    c.stream = stream;
    c.sigs = &hdr->sig;
    c.io = &hdr->io;
    c.n_sigs = 1;
    c.synd = base + kOffSynd;
    c.fp64 = fp64;
    c.in_fp64 = in64;
    c.epart = (double*)(base + kOffEpart);
    c.sigma = (double*)(base + kOffSigma);
    c.ebin = (double*)(base + kOffEbin);
    c.prechk = nullptr;   // general mode only
    c.sel = (SelDev*)(base + kOffSel);
    c.cnt = (SigCounters*)(base + kOffCnt);
    c.st_loc = (int64_t*)(base + kOffStLoc);
    c.st_val = (double2*)(base + kOffStVal);
    c.shifts = hdr->shifts;
    c.twiddle = fp64 ? (const void*)(base + kOffTw64) : (const void*)(base + kOffTw32);
    c.tw_log2 = fp64 ? kNaTw64Log2 : kNaTw32Log2;
    c.omega = (const double2*)(base + kOffOmega);
    c.gram = nullptr;
    c.om_log2 = kNaOmLog2;
    if (small) {
        c.synd_small_items = hdr->synd_items;
        c.n_synd_small_items = n_synd;
    } else {
        c.synd_items = hdr->synd_items;
        c.n_synd_items = n_synd;
    }
    if (pb) {
        const int grp = pair_group(pb, ilog2_na(g.m));
        c.pair_items = hdr->pair_items;
        c.pair_off[grp] = 0;
        c.pair_n[grp] = n_pair;
    }
    c.bin_items = hdr->bin_items;
    c.n_bin_items = n_bins;
    c.act_items = hdr->act_items;
    c.n_act_items = n_act;
    c.max_l = g.L;
    c.kidx = (int*)(base + kOffKidx);
    c.rk_a = (double*)(base + kOffRkA);
    c.rk_b = (long long*)(base + kOffRkB);
    c.rk_i = (int*)(base + kOffRkI);
    c.rk_r = (int*)(base + kOffRkR);
    c.work = (WorkCounters*)(base + kOffWork);
    c.active_list = (int2*)(base + kOffActive);
    c.qlist = (int2*)(base + kOffQlist);
    c.list_cap = g.m;
    c.n_work_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g.m + kBlock - 1) / kBlock, 1024));
    return enqueue_path(c, nullptr, nullptr, nullptr);
}
