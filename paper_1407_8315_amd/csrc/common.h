// Internal declarations of the sFFT-DT device library (gfx950).
//
// Layout in HBM (per plan; offsets are per signal and live in SigDev):
//   syndromes  [sig][k][2L]     the 2L consecutive shifts of bin k side by side
//                               (64 B per bin for complex64 input and L = 4),
//                               so that the lane-per-bin decoder, which takes
//                               bins in queue order, fetches each as one run;
//              [sig][R][k]      general mode: the R random shifts n_j by line;
//                               complex float for complex64 input, complex
//                               double for complex128.  Iterative grids keep
//                               [line][k] (synd_at()).
//   epart      [sig][line]      sum_k |m_l[k]|^2 (FP64), for mean_k E_k
//   sigma      [sig][k][L]      Hankel singular values (general mode)
//   ebin       [sig][k]         E_k (general mode)
//   staging    [sig][M*L]       (location, value) pairs appended by the decoder
//   counters   [sig]            SigCounters
// Iterative mode (Alg. 1) keeps, per signal, the syndromes of iteration l as
// the two lines of "view" l (a SigDev entry of its own, after the signals,
// with the d, M, offsets and table stride of that iteration's grid), and
//   status     [sig][l][k]      0 inactive, 1 solved, 2 failed (uint8)
//   records    [sig][l][k][l+1] (location, value, staging slot) of the
//                               frequencies a solved bin holds (SubFreq of
//                               later iterations; corrections of a location
//                               accumulate in its first staging slot)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sft {

constexpr int kMaxL = 4;
constexpr int kMaxLines = 2 * kMaxL + 64;   // 2L consecutive + up to 64 random shifts
constexpr int kBlock = 256;                 // threads per block of every kernel but select
constexpr int kFftPointsF32 = 8192;         // points per block in LDS (64 KiB)
constexpr int kFftPointsF64 = 4096;
constexpr int kFftPointsF32Small = 4096;     // blocks of FP32 signals with M <= this (32 KiB)
constexpr int kActivityTile = 4096;         // bins per block of the activity pass
// Consecutive-shift line pairs (pair_syndrome_kernel): FP32 units with
// 2^kPairLog2MMin <= M <= 2^kPairLog2MMax, P = 1, 2 or 4 pairs per block; one
// item list per (P, log2 M) group.  P = 0: iterative signals whose grids
// all qualify, every grid of a signal in one launch (iter_pair_kernel, by
// log2 M_0).
constexpr int kPairLog2MMin = 8, kPairLog2MMax = 12;
// log2 of the points of each line a thread holds (8: 107 VGPRs at M = 4096,
// four waves per SIMD; 16 points need 177 and measured 1.13x slower)
constexpr int kPairLpt = 3;
constexpr int kPairSizes = kPairLog2MMax - kPairLog2MMin + 1;
constexpr int kPairGroups = 4 * kPairSizes;
__host__ __device__ constexpr int pair_group(int p, int log2m) {
    return (p == 1 ? 0 : p == 2 ? 1 : p == 4 ? 2 : 3) * kPairSizes + (log2m - kPairLog2MMin);
}

enum Mode { kExact = 0, kGeneral = 1, kIterative = 2 };
constexpr int kFlagSpAll = 32;   // SFT_FLAG_SP_ALL (sft.h)

// Per-signal description, built by the plan and read by every kernel.
struct SigDev {
    int64_t n, d;            // N, d = N / M
    int32_t m, log2m;        // M
    int32_t L, R, S;         // max order, random shifts, lines = 2L (+ R)
    int32_t mode, k_votes;   // Mode, K (general mode vote / output size)
    int32_t flags;
    int64_t synd_off;        // element offset of [S][M] in the syndrome buffer
    int64_t epart_off;       // offset of [S] in epart
    int64_t bin_off;         // offset of [M] per-bin arrays (sigma uses bin_off * L)
    int64_t stage_off;       // offset of the staging list
    int32_t stage_cap;       // = M * L
    int32_t shift_off;       // offset of the S shift values in the shift table
    int32_t tab_stride;      // omega table stride: w_d^q = tab[q * tab_stride]
    int32_t log2m1;          // two-pass FFT (M above one block): M = M1 * M2, log2 M1 (0: one pass)
    int32_t bstride;         // syndromes of the 2L consecutive shifts by bin, [M][bstride] (bstride = 2L);
                             // 0: every line by line, [S][M] (iterative grids)
    int64_t rnd_off;         // general mode: element offset of the random shifts' [R][M] syndromes
    int64_t y_off;           // two-pass FFT: offset of the [S][M2][M1] intermediate
    int32_t parent;          // signal whose input and counters this entry uses (itself, or the owner of a view)
    int32_t view0;           // iterative mode: index of the view of iteration 0
    int64_t it_st_off;       // iterative mode: offset of the signal's status bytes
    int64_t it_rec_off;      // iterative mode: offset of the signal's records
    int64_t gram_off;        // general mode: offset of the signal's Gram row table F[0 .. d) (CS step)
    double tau_zero2, tau_rank, tau_res2, tau_amp, c_res, delta_grid, delta_mag;
};

// Element index of syndrome (line, k) of a unit in the syndrome buffer.  The
// non-iterative path keeps a bin's 2L consecutive-shift syndromes side by side
// (the kernels that follow the FFTs take one bin per lane, in queue order,
// and fetch them as one 64-byte run); the random shifts of general mode,
// written by one FFT block per line and read by the CS step only, and the
// lines of iterative grids stay by line.
__host__ __device__ inline int64_t synd_at(const SigDev& u, int line, int64_t k) {
    if (u.bstride == 0) return u.synd_off + ((int64_t)line << u.log2m) + k;
    if (line < u.bstride) return u.synd_off + k * u.bstride + line;
    return u.rnd_off + ((int64_t)(line - u.bstride) << u.log2m) + k;
}

// Per-call input/output pointers of a signal.
struct IoDev {
    const void* x;
    int64_t* loc;
    double2* val;
    int64_t cap;
    int64_t* count;
};

// Iterative mode: bins of iterations 0 .. l-1 (M_0 + M_0/2 + ...), and their
// records ((l'+1) per bin of iteration l').
__host__ __device__ inline int64_t iter_bins_off(int64_t m0, int l) { return 2 * m0 - ((2 * m0) >> l); }
__host__ __device__ inline int64_t iter_rec_off(int64_t m0, int l) {
    int64_t off = 0;
    for (int i = 0; i < l; ++i) off += (m0 >> i) * (i + 1);
    return off;
}

struct SigCounters {
    int stage_count, active, flagged, cs, mlp_fb, nonfinite, kept, pad;
    int it_queued[kMaxL];   // iterative mode: bins queued for SynDec in iteration l (own region per signal)
    int pad2[kMaxL];
};

// Plan-wide work lists, rebuilt by every call.  The decoder runs in rounds:
// round r tries the r-th hypothesis of every bin still open, with one kernel
// per order a, so that each kernel carries the code of one order only.  Two
// sets of round queues alternate (round r reads set r % 2 and fills set
// (r + 1) % 2); slot 0 of a set holds bins waiting for the rank test, slot a
// the bins whose next hypothesis has order a.  Flagged bins of general-mode
// signals end in the CS queue of their vote order.  Besides these, the active
// list holds the active bins of exact-mode signals (rank test or predictor
// input).
// The rank test itself runs in two passes: a certificate pass settles the
// rank-one bins (and tries their order 1 at once) and queues the others as
// pending, for the SVD pass (or, in a learned plan, for the predictor).
// In plans with general-mode signals, orders 3 and 4 (root finding by
// iteration) also run in two passes per round: the locator and |c_0| check
// for every bin, then the roots, grid check and judge for the survivors,
// queued per set in the roots queues.
constexpr int kRoundSlots = kMaxL + 1;
constexpr int kQueues = 2 * kRoundSlots + kMaxL + 1 + 4;
__host__ __device__ constexpr int q_round(int set, int slot) { return set * kRoundSlots + slot; }
__host__ __device__ constexpr int q_cs(int a0) { return 2 * kRoundSlots + a0 - 1; }
constexpr int kQPending = 2 * kRoundSlots + kMaxL;
__host__ __device__ constexpr int q_roots(int set, int a) { return kQPending + 1 + set * 2 + (a - 3); }

struct WorkCounters {
    int n_active;
    int q[kQueues];   // lengths of the queues above
};
static_assert(sizeof(WorkCounters) == (1 + kQueues) * sizeof(int), "WorkCounters: the active count and the queues");

// A list entry is (signal, code): code = k << 9 | step << 6 | ap << 3 | a0 with
// bin k (< 2^22), index `step` of the bin's next hypothesis in its order
// sequence, learned order ap (0: none) and rank-test or vote order a0 (0: not
// known yet).  CS queue entries are (signal, k).
__host__ __device__ inline int pack_code(int64_t k, int step, int ap, int a0) {
    return (int)(k << 9) | (step << 6) | (ap << 3) | a0;
}
__host__ __device__ inline int code_k(int c) { return c >> 9; }
__host__ __device__ inline int code_step(int c) { return (c >> 6) & 7; }
__host__ __device__ inline int code_ap(int c) { return (c >> 3) & 7; }
__host__ __device__ inline int code_a0(int c) { return c & 7; }

struct SelDev {             // per-signal results of the selection pass (general mode)
    unsigned long long thr_key;   // K-th largest singular value (as ordered bits)
    long long thr_idx;            // ties at thr_key vote when flat index <= thr_idx
    double nu;                    // noise floor
    double pad;
};

// Queue kQueues is the active list; the others are the round and CS queues.
__device__ inline int* queue_counter(WorkCounters* w, int q) { return q == kQueues ? &w->n_active : &w->q[q]; }
__device__ inline int2* queue_list(int2* active, int2* qlist, int64_t cap, int q) {
    return q == kQueues ? active : qlist + (int64_t)q * cap;
}

// Block-aggregated appends: in each trip of a block-uniform loop every thread
// calls reserve() with its target queue (or -1), then commit() writes the
// entries with one global atomic per non-empty queue and block.
struct BlockQueues {
    int cnt[kQueues + 1];
    int base[kQueues + 1];
    __device__ void reset() {
        if (threadIdx.x <= kQueues) cnt[threadIdx.x] = 0;
        __syncthreads();
    }
    __device__ int reserve(int q) { return q >= 0 ? atomicAdd(&cnt[q], 1) : 0; }
    __device__ void commit(WorkCounters* w, int2* active, int2* qlist, int64_t cap, int q, int slot, int2 ent) {
        __syncthreads();
        if (threadIdx.x <= kQueues && cnt[threadIdx.x] > 0) base[threadIdx.x] = atomicAdd(queue_counter(w, threadIdx.x), cnt[threadIdx.x]);
        __syncthreads();
        if (q >= 0) queue_list(active, qlist, cap, q)[base[q] + slot] = ent;
        __syncthreads();
    }
};

// ---------------------------------------------------------------- complex FP64

struct zd {
    double x, y;
};
__host__ __device__ inline zd mk(double a, double b) { return zd{a, b}; }
__host__ __device__ inline zd operator+(zd a, zd b) { return zd{a.x + b.x, a.y + b.y}; }
__host__ __device__ inline zd operator-(zd a, zd b) { return zd{a.x - b.x, a.y - b.y}; }
__host__ __device__ inline zd operator-(zd a) { return zd{-a.x, -a.y}; }
__host__ __device__ inline zd operator*(zd a, zd b) { return zd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline zd operator*(double s, zd a) { return zd{s * a.x, s * a.y}; }
__host__ __device__ inline zd conj(zd a) { return zd{a.x, -a.y}; }
__host__ __device__ inline double norm2(zd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double cabs(zd a) { return sqrt(norm2(a)); }
__host__ __device__ inline zd cmul_conj(zd a, zd b) { return conj(a) * b; }   // conj(a) * b
// 1/x: on the device the hardware reciprocal refined by two Newton steps
// (within an ulp or two of the quotient; 1/0 and 1/inf give NaN instead of
// inf and 0, which the decoder's finiteness checks reject like the quotients
// they feed), on the host the IEEE division.
__host__ __device__ inline double frcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    return fma(fma(-x, y, 1.0), y, y);
#else
    return 1.0 / x;
#endif
}
__host__ __device__ inline zd cdiv(zd a, zd b) {
    // Smith's algorithm, one reciprocal of the scaled denominator
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y * frcp(b.x), inv = frcp(b.x + b.y * r);
        return zd{(a.x + a.y * r) * inv, (a.y - a.x * r) * inv};
    }
    const double r = b.x * frcp(b.y), inv = frcp(b.x * r + b.y);
    return zd{(a.x * r + a.y) * inv, (a.y * r - a.x) * inv};
}
__host__ __device__ inline zd csqrt(zd a) {
    double r = hypot(a.x, a.y);
    if (r == 0.0) return zd{0.0, 0.0};
    if (a.x >= 0.0) {
        double t = sqrt(0.5 * (r + a.x));
        return zd{t, a.y / (2.0 * t)};
    }
    double t = sqrt(0.5 * (r - a.x));
    return zd{fabs(a.y) / (2.0 * t), copysign(t, a.y)};
}
__host__ __device__ inline bool cfinite(zd a) { return __builtin_isfinite(a.x) && __builtin_isfinite(a.y); }

// e^{i 2 pi q / n} for an integer phase 0 <= q < n, n a power of two.
__device__ inline zd unit_root(int64_t q, int64_t n) {
    double s, c;
    // n a power of two: 2/n and q * (2/n) are exact, the same value as 2q/n
    // without a division per call
    sincospi((double)q * (2.0 / (double)n), &s, &c);
    return zd{c, s};
}

// ---------------------------------------------------------------- host launchers
// Defined in the .hip translation units; called by the C ABI layer.

struct LaunchCtx {
    hipStream_t stream;
    const SigDev* sigs;
    const IoDev* io;
    int n_sigs;
    void* synd;              // float2* or double2*
    bool fp64;               // FFTs and syndromes in FP64
    bool in_fp64;            // complex128 input (else complex64)
    double* epart;
    double* sigma;
    double* ebin;
    unsigned char* prechk;   // general mode, per bin: round 0's |c_0| checks of orders 3, 4 (bit 0: taken)
    SelDev* sel;
    SigCounters* cnt;
    int64_t* st_loc;
    double2* st_val;
    const int64_t* shifts;
    const void* twiddle;     // float2* / double2* of size 2^tw_log2: e^{-2 pi i q / 2^tw_log2}
    int tw_log2;
    const double2* omega;    // e^{+2 pi i q / 2^om_log2}, FP64
    const double2* gram;     // general mode: Gram row tables F, indexed by SigDev::gram_off
    int om_log2;
    const int4* synd_items;  // (sig, line0, nlines, pass): pass 0 one-pass, 1 first of two
    int n_synd_items;
    const int4* synd_small_items;   // pass 0 items of FP32 signals with M <= kFftPointsF32Small
    int n_synd_small_items;
    const int4* synd_late_items;    // general mode's random-shift lines (pass 0), regular / small blocks
    int n_synd_late_items;
    const int4* synd_late_small_items;
    int n_synd_late_small_items;
    const int4* pair_items;  // (unit, line0, 0, 0): pair_syndrome_kernel blocks, grouped by pair_group()
    int pair_off[kPairGroups];
    int pair_n[kPairGroups];
    const int4* synd2_items; // second pass of two-pass signals (pass 2)
    int n_synd2_items;
    void* ybuf;              // two-pass intermediate (float2* / double2*)
    const int2* line_items;  // (sig, line) of two-pass signals, for the line energies
    int n_line_items;
    const int2* bin_items;   // (sig, bin0): tiles of kBlock bins
    int n_bin_items;
    const int2* act_items;   // (sig, bin0): tiles of kActivityTile bins
    int n_act_items;
    int n_general;           // signals in general mode
    const int* general_sigs; // their indices
    int any_general;
    int max_l;               // largest L of the plan's signals
    int* kidx;               // per staging entry: kept entries (output pass)
    double* rk_a;            // ranking scratch, one slot per staging entry
    long long* rk_b;
    int* rk_i;
    int* rk_r;
    WorkCounters* work;      // list lengths
    int2* active_list;       // [list_cap]
    int2* qlist;             // [kQueues][list_cap]: round queues, then CS queues
    int64_t list_cap;        // total bins of the plan
    int n_work_blocks;       // grid of the list-driven kernels
    // iterative mode (Alg. 1)
    bool iterative;
    uint8_t* it_status;
    int64_t* it_loc;
    double2* it_val;
    int* it_slot;
    const int2* it_items;            // (sig, bin0): tiles of kBlock bins, iteration by iteration
    int it_item_off[kMaxL];
    int it_n_items[kMaxL];
};

hipError_t launch_zero_counters(const LaunchCtx& c);
// sft_syndromes: unit 0's S lines into out as [S][M] (elems = S M)
hipError_t launch_copy_syndromes(const LaunchCtx& c, int64_t elems, void* out);
// part 0: every syndrome kernel; 1: all but the late items (general mode's
// random-shift lines); 2: the late items only
hipError_t launch_syndromes(const LaunchCtx& c, int part = 0);
hipError_t launch_singular_values(const LaunchCtx& c);
hipError_t launch_select(const LaunchCtx& c);
hipError_t launch_activity(const LaunchCtx& c);
hipError_t launch_certify(const LaunchCtx& c);                           // active list -> order 1 tried, or pending
hipError_t launch_svd_rank(const LaunchCtx& c, int q_in, int set_out);   // rank test by SVD
hipError_t launch_zero_set(const LaunchCtx& c, int set);
hipError_t launch_round(const LaunchCtx& c, int round, int a);   // the kernels of order a in round `round`
hipError_t launch_rest(const LaunchCtx& c);   // rounds 1.. in one kernel (plans without general-mode signals)
hipError_t launch_precheck(const LaunchCtx& c);   // general mode: round 0's pre-checks of orders 3 and 4
hipError_t launch_cs(const LaunchCtx& c, int a0);                // CS step of the bins flagged with vote order a0
hipError_t launch_output(const LaunchCtx& c);
hipError_t launch_iteration(const LaunchCtx& c, int l);   // Alg. 1, iteration l (scan, then SynDec for l >= 1)

}  // namespace sft
