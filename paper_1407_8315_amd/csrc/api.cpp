// C ABI of the sFFT-DT device library: plans, calls, status codes.
// The arithmetic of the method lives in fft.hip and decode.hip; this file
// validates parameters, chooses defaults, draws the random shifts, lays out
// the workspace, orders the work items and enqueues the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "plan_host.h"
#include "sft.h"

using namespace sft;

namespace {

thread_local std::string g_err;

sft_status fail(sft_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(SFT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct sft_plan_s {
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<SigHost> sig;
    bool fp64 = false;       // FFTs and syndromes in FP64
    bool in64 = false;       // complex128 input
    bool any_general = false;
    // device buffers
    std::vector<void*> allocs;
    SigDev* d_sigs = nullptr;
    IoDev* d_io = nullptr;
    void* d_synd = nullptr;
    double* d_epart = nullptr;
    double* d_sigma = nullptr;
    double* d_ebin = nullptr;
    unsigned char* d_prechk = nullptr;
    SelDev* d_sel = nullptr;
    SigCounters* d_cnt = nullptr;
    int64_t* d_stloc = nullptr;
    double2* d_stval = nullptr;
    int* d_kidx = nullptr;
    double* d_rk_a = nullptr;
    long long* d_rk_b = nullptr;
    int* d_rk_i = nullptr;
    int* d_rk_r = nullptr;
    int64_t* d_shifts = nullptr;
    void* d_tw = nullptr;
    double2* d_om = nullptr;
    double2* d_gram = nullptr;
    int4* d_synd_items = nullptr;
    int4* d_synd_small_items = nullptr;
    int n_synd_small_items = 0;
    int4* d_synd_late_items = nullptr;
    int4* d_synd_late_small_items = nullptr;
    int n_synd_late_items = 0, n_synd_late_small_items = 0;
    int4* d_synd2_items = nullptr;
    int4* d_pair_items = nullptr;
    int pair_off[kPairGroups] = {};
    int pair_n[kPairGroups] = {};
    int2* d_line_items = nullptr;
    void* d_ybuf = nullptr;
    int n_synd2_items = 0, n_line_items = 0;
    int2* d_bin_items = nullptr;
    int2* d_act_items = nullptr;
    int* d_gsigs = nullptr;
    bool iterative = false;          // Alg. 1 plan
    uint8_t* d_it_status = nullptr;
    int64_t* d_it_loc = nullptr;
    double2* d_it_val = nullptr;
    int* d_it_slot = nullptr;
    int2* d_it_items = nullptr;
    int it_item_off[kMaxL] = {0, 0, 0, 0};
    int it_n_items[kMaxL] = {0, 0, 0, 0};
    WorkCounters* d_work = nullptr;
    int2* d_active = nullptr;
    int2* d_qlist = nullptr;
    int max_l = 1;
    int64_t list_cap = 0;
    int n_work_blocks = 0;
    int n_synd_items = 0, n_bin_items = 0, n_act_items = 0, n_general = 0;
    int tw_log2 = 0, om_log2 = 0;
    int64_t ws_bytes = 0;
    // host staging
    IoDev* h_io = nullptr;
    std::vector<IoDev> dev_io;   // the table the device holds (valid when io_valid)
    bool io_valid = false;
    SigCounters* h_cnt = nullptr;
    hipEvent_t ev_upload = nullptr;
    bool upload_pending = false;
    // stage boundaries of timed calls; ev[5]: between the consecutive-shift
    // and the random-shift gathers
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // branches for independent kernels of one stage (the orders of a round,
    // the CS orders): default-priority streams, forked from and joined into
    // the plan's stream with events (captured into the graph as parallel
    // branches)
    hipStream_t side[kMaxL - 1] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipStream_t late = nullptr;   // general mode: random-shift lines beside the rounds
    hipEvent_t ev_late_fork = nullptr, ev_late_join = nullptr;
    hipEvent_t ev_join[kMaxL - 1] = {nullptr, nullptr, nullptr};
    sft_mlp_t mlp = nullptr;
    std::vector<sft_plan_s*> rungs;   // unknown K: plans of the smaller M, ascending (this plan is the last rung)
};

namespace {

template <typename T>
sft_status dalloc(sft_plan_s* p, T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) return fail(SFT_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->allocs.push_back(ptr);
    p->ws_bytes += (int64_t)(count * sizeof(T));
    *out = (T*)ptr;
    return SFT_OK;
}

void release(sft_plan_s* p) {
    if (!p) return;
    for (sft_plan_s* r : p->rungs) release(r);
    p->rungs.clear();
    if (p->stream || true) (void)hipStreamSynchronize(p->stream);
    for (void* a : p->allocs) (void)hipFree(a);
    p->allocs.clear();
    if (p->h_io) (void)hipHostFree(p->h_io);
    if (p->h_cnt) (void)hipHostFree(p->h_cnt);
    if (p->ev_upload) (void)hipEventDestroy(p->ev_upload);
    for (auto& e : p->ev)
        if (e) (void)hipEventDestroy(e);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto& st : p->side)
        if (st) (void)hipStreamDestroy(st);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->late) (void)hipStreamDestroy(p->late);
    if (p->ev_late_fork) (void)hipEventDestroy(p->ev_late_fork);
    if (p->ev_late_join) (void)hipEventDestroy(p->ev_late_join);
    for (auto& e : p->ev_join)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

LaunchCtx make_ctx(const sft_plan_s* p) {
    LaunchCtx c{};
    c.stream = p->stream;
    c.sigs = p->d_sigs;
    c.io = p->d_io;
    c.n_sigs = (int)p->sig.size();
    c.synd = p->d_synd;
    c.fp64 = p->fp64;
    c.in_fp64 = p->in64;
    c.epart = p->d_epart;
    c.sigma = p->d_sigma;
    c.ebin = p->d_ebin;
    c.prechk = p->d_prechk;
    c.sel = p->d_sel;
    c.cnt = p->d_cnt;
    c.st_loc = p->d_stloc;
    c.st_val = p->d_stval;
    c.shifts = p->d_shifts;
    c.twiddle = p->d_tw;
    c.tw_log2 = p->tw_log2;
    c.omega = p->d_om;
    c.gram = p->d_gram;
    c.om_log2 = p->om_log2;
    c.synd_items = p->d_synd_items;
    c.n_synd_items = p->n_synd_items;
    c.synd_small_items = p->d_synd_small_items;
    c.n_synd_small_items = p->n_synd_small_items;
    c.synd_late_items = p->d_synd_late_items;
    c.n_synd_late_items = p->n_synd_late_items;
    c.synd_late_small_items = p->d_synd_late_small_items;
    c.n_synd_late_small_items = p->n_synd_late_small_items;
    c.pair_items = p->d_pair_items;
    for (int g = 0; g < kPairGroups; ++g) {
        c.pair_off[g] = p->pair_off[g];
        c.pair_n[g] = p->pair_n[g];
    }
    c.synd2_items = p->d_synd2_items;
    c.n_synd2_items = p->n_synd2_items;
    c.ybuf = p->d_ybuf;
    c.line_items = p->d_line_items;
    c.n_line_items = p->n_line_items;
    c.bin_items = p->d_bin_items;
    c.n_bin_items = p->n_bin_items;
    c.act_items = p->d_act_items;
    c.n_act_items = p->n_act_items;
    c.n_general = p->n_general;
    c.general_sigs = p->d_gsigs;
    c.any_general = p->any_general ? 1 : 0;
    c.max_l = p->max_l;
    c.kidx = p->d_kidx;
    c.rk_a = p->d_rk_a;
    c.rk_b = p->d_rk_b;
    c.rk_i = p->d_rk_i;
    c.rk_r = p->d_rk_r;
    c.work = p->d_work;
    c.active_list = p->d_active;
    c.qlist = p->d_qlist;
    c.list_cap = p->list_cap;
    c.n_work_blocks = p->n_work_blocks;
    c.iterative = p->iterative;
    c.it_status = p->d_it_status;
    c.it_loc = p->d_it_loc;
    c.it_val = p->d_it_val;
    c.it_slot = p->d_it_slot;
    c.it_items = p->d_it_items;
    for (int l = 0; l < kMaxL; ++l) {
        c.it_item_off[l] = p->it_item_off[l];
        c.it_n_items[l] = p->it_n_items[l];
    }
    return c;
}

bool learned(const sft_plan_s* p) {
    for (auto& g : p->sig)
        if (g.flags & SFT_FLAG_LEARNED) return true;
    return false;
}

}  // namespace

namespace sft {

sft_status set_error(sft_status s, const std::string& msg) { return fail(s, msg); }

// Run fn(ctx, i) for i = 1..n as parallel branches after everything already
// enqueued on c.stream: branch 1 on c.stream itself, branch i > 1 on side
// stream i-2 (a process has few hardware queues, so the main stream carries
// one branch); c.stream then waits for all.  Without br, in series.
template <typename Fn>
static sft_status branches(const Branching* br, const LaunchCtx& c, int n, Fn fn) {
    if (n <= 1 || !br) {
        for (int i = 1; i <= n; ++i) HIPCHK(fn(c, i));
        return SFT_OK;
    }
    HIPCHK(hipEventRecord(br->fork, c.stream));
    for (int i = 1; i < n; ++i) {
        HIPCHK(hipStreamWaitEvent(br->side[i - 1], br->fork, 0));
        LaunchCtx ci = c;
        ci.stream = br->side[i - 1];
        HIPCHK(fn(ci, i + 1));
        HIPCHK(hipEventRecord(br->join[i - 1], br->side[i - 1]));
    }
    HIPCHK(fn(c, 1));
    for (int i = 1; i < n; ++i) HIPCHK(hipStreamWaitEvent(c.stream, br->join[i - 1], 0));
    return SFT_OK;
}

sft_status enqueue_path(const LaunchCtx& c, const Branching* br, sft_mlp_t mlp, hipEvent_t* events) {
    const bool use_mlp = mlp != nullptr;
    const bool any_exact = c.n_general < c.n_sigs;
    HIPCHK(launch_zero_counters(c));
    if (events) HIPCHK(hipEventRecord(events[0], c.stream));
    // General mode's random-shift lines, which only the CS step reads, start
    // on a stream of their own right after the other lines, beside the order
    // estimate and the rounds, and join the main stream before the CS step
    // (started later, after the singular values or the selection, they take
    // the CUs of the kernel launched next and measured slower).  Timed calls
    // keep the stages in order.
    const bool late = (c.n_synd_late_items + c.n_synd_late_small_items) > 0 && br && br->late && !events;
    if (late) {
        HIPCHK(launch_syndromes(c, 1));
        HIPCHK(hipEventRecord(br->late_fork, c.stream));
        HIPCHK(hipStreamWaitEvent(br->late, br->late_fork, 0));
        LaunchCtx cl = c;
        cl.stream = br->late;
        HIPCHK(launch_syndromes(cl, 2));
        HIPCHK(hipEventRecord(br->late_join, br->late));
    } else if (events && c.n_synd_late_items + c.n_synd_late_small_items > 0) {
        // timed: the random-shift lines after the others, each part timed
        HIPCHK(launch_syndromes(c, 1));
        HIPCHK(hipEventRecord(events[5], c.stream));
        HIPCHK(launch_syndromes(c, 2));
    } else {
        HIPCHK(launch_syndromes(c));
    }
    if (events) HIPCHK(hipEventRecord(events[1], c.stream));
    HIPCHK(launch_singular_values(c));
    HIPCHK(launch_select(c));
    HIPCHK(launch_activity(c));
    // Round-0 queues: general-mode bins come from the vote (activity pass).
    // Exact-mode bins go through the rank test: the certificate pass settles
    // the rank-one bins (and tries order 1 on them at once); the pending ones
    // get the SVD pass, or in a learned plan the predictor, with the SVD pass
    // for the bins it gives no order.
    if (any_exact) {
        HIPCHK(launch_certify(c));
        if (use_mlp) {
            sft_status s = sft_mlp_launch_infer(mlp, c);
            if (s != SFT_OK) return s;
            // bins without a predicted order: in plans with general-mode
            // signals the SVD pass now, otherwise the rest kernel's rank test
            if (c.n_general > 0) HIPCHK(launch_svd_rank(c, q_round(0, 0), 0));
        } else {
            HIPCHK(launch_svd_rank(c, kQPending, 0));
        }
    }
    if (events) HIPCHK(hipEventRecord(events[2], c.stream));
    for (int r = 0; r < c.max_l; ++r) {
        if (r >= 1) HIPCHK(launch_zero_set(c, (r + 1) & 1));
        // the orders of a round read their own queues: parallel branches
        const int n_orders = (r == 0 && !c.any_general) ? std::min(c.max_l, 2) : c.max_l;
        // round 0 of general mode: the pre-checks of orders 3 and 4 for the
        // later rounds, after the short order-2 kernel in its branch
        sft_status bs = branches(br, c, n_orders, [&](const LaunchCtx& ci, int a) {
            hipError_t e = launch_round(ci, r, a);
            if (e == hipSuccess && r == 0 && a == 2 && c.any_general) e = launch_precheck(ci);
            return e;
        });
        if (bs != SFT_OK) return bs;
        // bins whose learned order failed: rank test, then on with round 1
        // (without general-mode signals the rest kernel runs it itself)
        if (r == 0 && use_mlp && c.max_l > 1 && c.n_general > 0) HIPCHK(launch_svd_rank(c, q_round(1, 0), 1));
        // without general-mode signals, the few bins left after round 0 of orders 1
        // and 2 finish in one kernel
        if (r == 0 && c.n_general == 0 && c.max_l > 1) {
            HIPCHK(launch_rest(c));
            break;
        }
    }
    if (late) HIPCHK(hipStreamWaitEvent(c.stream, br->late_join, 0));
    if (c.any_general) {
        // one branch per order: order 1 on the main stream, then the rare
        // orders 3 and 4, then order 2 (with four hardware queues per process,
        // the runtime can run two branches on one queue, in series; measured,
        // the first two side branches share one, so they carry the cheap pair)
        static constexpr int kCsOrder[kMaxL] = {1, 3, 4, 2};
        sft_status bs = branches(br, c, kMaxL, [&](const LaunchCtx& ci, int b) { return launch_cs(ci, kCsOrder[b - 1]); });
        if (bs != SFT_OK) return bs;
    }
    if (events) HIPCHK(hipEventRecord(events[3], c.stream));
    HIPCHK(launch_output(c));
    if (events) HIPCHK(hipEventRecord(events[4], c.stream));
    return SFT_OK;
}

}  // namespace sft

namespace {

// Enqueue the whole path.  With events != nullptr, record stage boundaries.
// Learned plans run the predictor between the activity pass and the decoder.
sft_status enqueue(const sft_plan_s* p, hipEvent_t* events) {
    LaunchCtx c = make_ctx(p);
    if (p->iterative) {
        // Alg. 1: the FFTs of every iteration in one stage (they depend on x
        // only), then the iterations in order, then the output pass
        HIPCHK(launch_zero_counters(c));
        if (events) HIPCHK(hipEventRecord(events[0], p->stream));
        HIPCHK(launch_syndromes(c));
        if (events) HIPCHK(hipEventRecord(events[1], p->stream));
        for (int l = 0; l < p->max_l; ++l) {
            HIPCHK(launch_iteration(c, l));
            if (l == 0 && events) HIPCHK(hipEventRecord(events[2], p->stream));
        }
        if (events) HIPCHK(hipEventRecord(events[3], p->stream));
        HIPCHK(launch_output(c));
        if (events) HIPCHK(hipEventRecord(events[4], p->stream));
        return SFT_OK;
    }
    Branching br{};
    for (int i = 0; i < kMaxL - 1; ++i) {
        br.side[i] = p->side[i];
        br.join[i] = p->ev_join[i];
    }
    br.fork = p->ev_fork;
    br.late = p->late;
    br.late_fork = p->ev_late_fork;
    br.late_join = p->ev_late_join;
    return enqueue_path(c, &br, learned(p) ? p->mlp : nullptr, events);
}

sft_status upload_io(sft_plan_s* p, const void* const* xs, const sft_sparse_out* outs) {
    const size_t n = p->sig.size();
    for (size_t i = 0; i < n; ++i) {
        if (!xs[i]) return fail(SFT_E_INVALID, "input pointer is NULL (signal " + std::to_string(i) + ")");
        const sft_sparse_out& o = outs[i];
        if (!o.count_dev || o.capacity < 0 || (o.capacity > 0 && (!o.loc_dev || !o.val_dev)))
            return fail(SFT_E_INVALID, "output list is incomplete (signal " + std::to_string(i) + ")");
    }
    std::vector<IoDev> cur(n);
    for (size_t i = 0; i < n; ++i)
        cur[i] = IoDev{xs[i], outs[i].loc_dev, (double2*)outs[i].val_dev, outs[i].capacity, outs[i].count_dev};
    // repeated calls on the same buffers: the device already holds this table
    if (p->io_valid && std::memcmp(cur.data(), p->dev_io.data(), n * sizeof(IoDev)) == 0) return SFT_OK;
    if (p->upload_pending) HIPCHK(hipEventSynchronize(p->ev_upload));
    std::memcpy(p->h_io, cur.data(), n * sizeof(IoDev));
    HIPCHK(hipMemcpyAsync(p->d_io, p->h_io, n * sizeof(IoDev), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipEventRecord(p->ev_upload, p->stream));
    p->upload_pending = true;
    p->dev_io.swap(cur);
    p->io_valid = true;
    return SFT_OK;
}

// Wait, read the counters, fill stats, derive the status.
sft_status finish(sft_plan_s* p, sft_stats* st, bool timed) {
    const size_t n = p->sig.size();
    HIPCHK(hipMemcpyAsync(p->h_cnt, p->d_cnt, n * sizeof(SigCounters), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    HIPCHK(hipGetLastError());
    sft_stats s{};
    for (size_t i = 0; i < n; ++i) {
        const SigCounters& c = p->h_cnt[i];
        s.active_bins += c.active;
        s.flagged_bins += c.flagged;
        s.cs_bins += c.cs;
        s.mlp_fallbacks += c.mlp_fb;
        s.entries += c.kept;
        s.nonfinite += c.nonfinite;
        if (c.kept > p->h_io[i].cap) s.overflowed += 1;
    }
    for (int i = 0; i < 4; ++i) s.stage_ms[i] = -1.0;
    s.gather_ms[0] = s.gather_ms[1] = -1.0;
    if (timed) {
        for (int i = 0; i < 4; ++i) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
            s.stage_ms[i] = ms;
        }
        if (!p->iterative && p->n_synd_late_items + p->n_synd_late_small_items > 0) {
            float a = 0.f, b = 0.f;
            HIPCHK(hipEventElapsedTime(&a, p->ev[0], p->ev[5]));
            HIPCHK(hipEventElapsedTime(&b, p->ev[5], p->ev[1]));
            s.gather_ms[0] = a;
            s.gather_ms[1] = b;
        } else {
            s.gather_ms[0] = s.stage_ms[0];
            s.gather_ms[1] = 0.0;
        }
    }
    if (st) *st = s;
    if (s.nonfinite > 0) {
        bool check = false;
        for (auto& g : p->sig) check |= (g.flags & SFT_FLAG_CHECK_FINITE) != 0;
        if (check) return fail(SFT_E_NONFINITE, std::to_string(s.nonfinite) + " non-finite input samples gathered");
    }
    if (s.overflowed > 0)
        return fail(SFT_E_CAPACITY, std::to_string(s.overflowed) + " output list(s) too small; count holds the size");
    return SFT_OK;
}

bool any_sync(const sft_plan_s* p) {
    for (auto& g : p->sig)
        if (g.flags & SFT_FLAG_SYNC) return true;
    return false;
}

sft_status run_single(sft_plan_t plan, const void* x, const sft_sparse_out* out, sft_stats* st, int mode) {
    if (!plan || !out) return fail(SFT_E_INVALID, "plan or output is NULL");
    if (plan->sig.size() != 1) return fail(SFT_E_INVALID, "batch plans run through sft_batch");
    if (plan->sig[0].mode != mode)
        return fail(SFT_E_INVALID, mode == kExact     ? "plan is not in SFT_MODE_EXACT"
                                   : mode == kGeneral ? "plan is not in SFT_MODE_GENERAL"
                                                      : "plan is not in SFT_MODE_ITERATIVE");
    if ((plan->sig[0].flags & SFT_FLAG_LEARNED) && !plan->mlp)
        return fail(SFT_E_INVALID, "SFT_FLAG_LEARNED without an attached predictor");
    const void* xs[1] = {x};
    sft_status s = upload_io(plan, xs, out);
    if (s != SFT_OK) return s;
    const bool timed = st != nullptr;
    s = enqueue(plan, timed ? plan->ev : nullptr);
    if (s != SFT_OK) return s;
    if (st || any_sync(plan)) return finish(plan, st, timed);
    return SFT_OK;
}

}  // namespace

extern "C" {

int32_t sft_abi_version(void) { return SFT_ABI_VERSION; }

sft_status sft_autotune(int64_t n, int64_t k, int32_t in_dtype, double target, int64_t* m_out, int32_t* l_out,
                        double* expected_recovery, double* model_us) {
    if (!m_out || !l_out) return fail(SFT_E_INVALID, "m_out and l_out must not be NULL");
    std::string msg;
    int l = 0;
    sft_status st = autotune(n, k, in_dtype, target, m_out, &l, expected_recovery, model_us, &msg);
    if (st != SFT_OK) return fail(st, msg);
    *l_out = l;
    return SFT_OK;
}

const char* sft_last_error(void) { return g_err.c_str(); }

const char* sft_status_str(sft_status s) {
    switch (s) {
        case SFT_OK: return "SFT_OK";
        case SFT_E_INVALID: return "SFT_E_INVALID";
        case SFT_E_UNSUPPORTED: return "SFT_E_UNSUPPORTED";
        case SFT_E_NOMEM: return "SFT_E_NOMEM";
        case SFT_E_DEVICE: return "SFT_E_DEVICE";
        case SFT_E_CAPACITY: return "SFT_E_CAPACITY";
        case SFT_E_NONFINITE: return "SFT_E_NONFINITE";
    }
    return "unknown status";
}

sft_status sft_plan(sft_plan_t* out, const sft_params* params, int64_t n_params, void* hip_stream) {
    if (!out) return fail(SFT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!params || n_params < 1) return fail(SFT_E_INVALID, "need at least one parameter set");
    if (n_params > (1 << 24)) return fail(SFT_E_UNSUPPORTED, "too many signals in one plan");
    std::vector<SigHost> sigs((size_t)n_params);
    std::string msg;
    for (int64_t i = 0; i < n_params; ++i) {
        sft_status s = resolve_params(params[i], n_params > 1, &sigs[(size_t)i], &msg);
        if (s != SFT_OK) return fail(s, "signal " + std::to_string(i) + ": " + msg);
    }
    for (auto& g : sigs)
        if (g.dtype != sigs[0].dtype) return fail(SFT_E_UNSUPPORTED, "all signals of a plan need one input dtype");
    for (auto& g : sigs)
        if ((g.flags & SFT_FLAG_FFT64) != (sigs[0].flags & SFT_FLAG_FFT64))
            return fail(SFT_E_UNSUPPORTED, "SFT_FLAG_FFT64 must be set on all signals of a plan or on none");
    for (auto& g : sigs)
        if ((g.mode == SFT_MODE_ITERATIVE) != (sigs[0].mode == SFT_MODE_ITERATIVE))
            return fail(SFT_E_UNSUPPORTED, "a plan's signals are all in SFT_MODE_ITERATIVE or none is");

    sft_plan_s* p = new sft_plan_s();
    p->stream = (hipStream_t)hip_stream;
    p->sig = std::move(sigs);
    p->in64 = p->sig[0].dtype == SFT_C128;
    p->fp64 = p->in64 || (p->sig[0].flags & SFT_FLAG_FFT64) != 0;
    if (hipGetDevice(&p->device) != hipSuccess) {
        release(p);
        return fail(SFT_E_DEVICE, "no HIP device");
    }
    PlanLayout lay;
    build_layout(p->sig, p->fp64, &lay);
    p->any_general = lay.n_general > 0;
    p->n_general = lay.n_general;
    p->tw_log2 = lay.tw_log2;
    p->om_log2 = lay.om_log2;
    p->n_synd_items = (int)lay.synd_items.size();
    p->n_synd_small_items = (int)lay.synd_small_items.size();
    p->n_synd_late_items = (int)lay.synd_late_items.size();
    p->n_synd_late_small_items = (int)lay.synd_late_small_items.size();
    p->n_synd2_items = (int)lay.synd2_items.size();
    for (int g = 0; g < kPairGroups; ++g) {
        p->pair_off[g] = lay.pair_off[g];
        p->pair_n[g] = lay.pair_n[g];
    }
    p->n_line_items = (int)lay.line_items.size();
    p->n_bin_items = (int)lay.bin_items.size();
    p->n_act_items = (int)lay.act_items.size();
    p->iterative = lay.n_iterative > 0;
    for (int l = 0; l < kMaxL; ++l) {
        p->it_item_off[l] = lay.it_item_off[l];
        p->it_n_items[l] = lay.it_n_items[l];
    }

    const size_t ns = p->sig.size();
    sft_status s = SFT_OK;
#define TRY(x)             \
    do {                   \
        s = (x);           \
        if (s != SFT_OK) { \
            release(p);    \
            return s;      \
        }                  \
    } while (0)
    TRY(dalloc(p, &p->d_sigs, lay.sigdev.size()));
    TRY(dalloc(p, &p->d_io, ns));
    if (p->fp64) {
        double2* t = nullptr;
        TRY(dalloc(p, &t, (size_t)lay.synd_elems));
        p->d_synd = t;
        double2* yb = nullptr;
        TRY(dalloc(p, &yb, (size_t)lay.y_elems));
        p->d_ybuf = yb;
        double2* tw = nullptr;
        TRY(dalloc(p, &tw, (size_t)1 << lay.tw_log2));
        p->d_tw = tw;
    } else {
        float2* t = nullptr;
        TRY(dalloc(p, &t, (size_t)lay.synd_elems));
        p->d_synd = t;
        float2* yb = nullptr;
        TRY(dalloc(p, &yb, (size_t)lay.y_elems));
        p->d_ybuf = yb;
        float2* tw = nullptr;
        TRY(dalloc(p, &tw, (size_t)1 << lay.tw_log2));
        p->d_tw = tw;
    }
    TRY(dalloc(p, &p->d_epart, (size_t)lay.epart_elems));
    TRY(dalloc(p, &p->d_sigma, lay.n_general ? (size_t)lay.sigma_elems : 1));
    TRY(dalloc(p, &p->d_ebin, lay.n_general ? (size_t)lay.bin_elems : 1));
    TRY(dalloc(p, &p->d_prechk, lay.n_general ? (size_t)lay.bin_elems : 1));
    TRY(dalloc(p, &p->d_sel, ns));
    TRY(dalloc(p, &p->d_cnt, ns));
    TRY(dalloc(p, &p->d_stloc, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_stval, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_kidx, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_rk_a, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_rk_b, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_rk_i, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_rk_r, (size_t)lay.stage_elems));
    TRY(dalloc(p, &p->d_shifts, lay.shifts.size()));
    TRY(dalloc(p, &p->d_om, (size_t)1 << lay.om_log2));
    TRY(dalloc(p, &p->d_gram, std::max<size_t>(1, lay.gram.size())));
    TRY(dalloc(p, &p->d_synd_items, lay.synd_items.size()));
    TRY(dalloc(p, &p->d_synd_small_items, lay.synd_small_items.size()));
    TRY(dalloc(p, &p->d_synd_late_items, lay.synd_late_items.size()));
    TRY(dalloc(p, &p->d_synd_late_small_items, lay.synd_late_small_items.size()));
    TRY(dalloc(p, &p->d_synd2_items, lay.synd2_items.size()));
    TRY(dalloc(p, &p->d_pair_items, lay.pair_items.size()));
    TRY(dalloc(p, &p->d_line_items, lay.line_items.size()));
    TRY(dalloc(p, &p->d_bin_items, lay.bin_items.size()));
    TRY(dalloc(p, &p->d_act_items, lay.act_items.size()));
    TRY(dalloc(p, &p->d_gsigs, lay.general_sigs.size()));
    TRY(dalloc(p, &p->d_it_status, (size_t)lay.it_st_elems));
    TRY(dalloc(p, &p->d_it_loc, (size_t)lay.it_rec_elems));
    TRY(dalloc(p, &p->d_it_val, (size_t)lay.it_rec_elems));
    TRY(dalloc(p, &p->d_it_slot, (size_t)lay.it_rec_elems));
    TRY(dalloc(p, &p->d_it_items, lay.it_items.size()));
    TRY(dalloc(p, &p->d_work, 1));
    TRY(dalloc(p, &p->d_active, (size_t)lay.bin_elems));
    TRY(dalloc(p, &p->d_qlist, (size_t)lay.bin_elems * kQueues));
    p->list_cap = lay.bin_elems;
    for (auto& g : p->sig) p->max_l = std::max(p->max_l, g.L);
    {
        // grid of the list-driven kernels (grid-stride loops): a few blocks per
        // CU, never more than the bins themselves need
        int64_t need = (lay.bin_elems + kBlock - 1) / kBlock;
        p->n_work_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(need, 1024));
    }

#define HIPTRY(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            release(p);                                                                                \
            return fail(SFT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));              \
        }                                                                                              \
    } while (0)
    HIPTRY(hipMemcpy(p->d_sigs, lay.sigdev.data(), lay.sigdev.size() * sizeof(SigDev), hipMemcpyHostToDevice));
    if (!lay.it_items.empty())
        HIPTRY(hipMemcpy(p->d_it_items, lay.it_items.data(), lay.it_items.size() * sizeof(int2), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(p->d_shifts, lay.shifts.data(), lay.shifts.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (p->fp64) {
        std::vector<double2> tw;
        twiddle_table_f64(lay.tw_log2, &tw);
        HIPTRY(hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
    } else {
        std::vector<float2> tw;
        twiddle_table_f32(lay.tw_log2, &tw);
        HIPTRY(hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
    HIPTRY(hipMemcpy(p->d_om, lay.omega.data(), lay.omega.size() * sizeof(double2), hipMemcpyHostToDevice));
    if (!lay.gram.empty())
        HIPTRY(hipMemcpy(p->d_gram, lay.gram.data(), lay.gram.size() * sizeof(double2), hipMemcpyHostToDevice));
    if (!lay.synd_items.empty())
        HIPTRY(hipMemcpy(p->d_synd_items, lay.synd_items.data(), lay.synd_items.size() * sizeof(int4), hipMemcpyHostToDevice));
    if (!lay.synd_small_items.empty())
        HIPTRY(hipMemcpy(p->d_synd_small_items, lay.synd_small_items.data(), lay.synd_small_items.size() * sizeof(int4),
                         hipMemcpyHostToDevice));
    if (!lay.synd_late_items.empty())
        HIPTRY(hipMemcpy(p->d_synd_late_items, lay.synd_late_items.data(), lay.synd_late_items.size() * sizeof(int4),
                         hipMemcpyHostToDevice));
    if (!lay.synd_late_small_items.empty())
        HIPTRY(hipMemcpy(p->d_synd_late_small_items, lay.synd_late_small_items.data(),
                         lay.synd_late_small_items.size() * sizeof(int4), hipMemcpyHostToDevice));
    if (!lay.pair_items.empty())
        HIPTRY(hipMemcpy(p->d_pair_items, lay.pair_items.data(), lay.pair_items.size() * sizeof(int4),
                         hipMemcpyHostToDevice));
    if (!lay.synd2_items.empty())
        HIPTRY(hipMemcpy(p->d_synd2_items, lay.synd2_items.data(), lay.synd2_items.size() * sizeof(int4),
                         hipMemcpyHostToDevice));
    if (!lay.line_items.empty())
        HIPTRY(hipMemcpy(p->d_line_items, lay.line_items.data(), lay.line_items.size() * sizeof(int2),
                         hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(p->d_bin_items, lay.bin_items.data(), lay.bin_items.size() * sizeof(int2), hipMemcpyHostToDevice));
    HIPTRY(hipMemcpy(p->d_act_items, lay.act_items.data(), lay.act_items.size() * sizeof(int2), hipMemcpyHostToDevice));
    if (!lay.general_sigs.empty())
        HIPTRY(hipMemcpy(p->d_gsigs, lay.general_sigs.data(), lay.general_sigs.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPTRY(hipMemset(p->d_cnt, 0, ns * sizeof(SigCounters)));
    HIPTRY(hipHostMalloc((void**)&p->h_io, ns * sizeof(IoDev), hipHostMallocDefault));
    HIPTRY(hipHostMalloc((void**)&p->h_cnt, ns * sizeof(SigCounters), hipHostMallocDefault));
    HIPTRY(hipEventCreateWithFlags(&p->ev_upload, hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    if (p->any_general) {
        HIPTRY(hipStreamCreateWithFlags(&p->late, hipStreamNonBlocking));
        HIPTRY(hipEventCreateWithFlags(&p->ev_late_fork, hipEventDisableTiming));
        HIPTRY(hipEventCreateWithFlags(&p->ev_late_join, hipEventDisableTiming));
    }
    for (auto& e : p->ev_join) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& st : p->side) HIPTRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (auto& e : p->ev) HIPTRY(hipEventCreate(&e));
    HIPTRY(hipDeviceSynchronize());
    if (p->sig[0].flags & SFT_FLAG_UNKNOWN_K) {
        // the rungs below this plan's M, each a plain single-signal plan
        const int64_t m_min = std::max<int64_t>(1, p->sig[0].n >> 22);
        for (int64_t m = m_min; m < p->sig[0].m; m *= 2) {
            sft_params q = params[0];
            q.m = m;
            q.flags &= ~(uint32_t)SFT_FLAG_UNKNOWN_K;
            sft_plan_t r = nullptr;
            sft_status rs = sft_plan(&r, &q, 1, hip_stream);
            if (rs != SFT_OK) {
                std::string msg = g_err;
                release(p);
                return fail(rs, "unknown-K rung M = " + std::to_string(m) + ": " + msg);
            }
            p->rungs.push_back(r);
        }
    }
    *out = p;
    return SFT_OK;
}

sft_status sft_exact(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats) {
    return run_single(plan, x_dev, out, stats, kExact);
}

sft_status sft_unknown_k(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats,
                         int64_t* m_chosen) {
    if (!plan || !out) return fail(SFT_E_INVALID, "plan or output is NULL");
    if (plan->sig.size() != 1 || !(plan->sig[0].flags & SFT_FLAG_UNKNOWN_K))
        return fail(SFT_E_INVALID, "plan was not created with SFT_FLAG_UNKNOWN_K");
    const size_t n_rungs = plan->rungs.size() + 1;
    for (size_t i = 0; i < n_rungs; ++i) {
        sft_plan_s* r = i + 1 < n_rungs ? plan->rungs[i] : plan;
        const bool last = i + 1 == n_rungs;
        sft_stats st{};
        sft_status s = run_single(r, x_dev, out, &st, kExact);
        if (s != SFT_OK && s != SFT_E_CAPACITY) return s;
        // an overflowing list only matters for the rung whose list is returned
        if (st.flagged_bins == 0 || last) {
            if (m_chosen) *m_chosen = r->sig[0].m;
            if (stats) *stats = st;
            return s;
        }
    }
    return SFT_OK;
}

sft_status sft_iterative(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats) {
    return run_single(plan, x_dev, out, stats, kIterative);
}

sft_status sft_general(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats) {
    return run_single(plan, x_dev, out, stats, kGeneral);
}

sft_status sft_batch(sft_plan_t plan, const void* const* x_devs, const sft_sparse_out* outs, sft_stats* stats) {
    if (!plan || !x_devs || !outs) return fail(SFT_E_INVALID, "plan, inputs or outputs is NULL");
    for (auto& g : plan->sig)
        if (g.flags & SFT_FLAG_LEARNED) {
            if (!plan->mlp) return fail(SFT_E_INVALID, "SFT_FLAG_LEARNED without an attached predictor");
        }
    sft_status s = upload_io(plan, x_devs, outs);
    if (s != SFT_OK) return s;
    if (stats) {
        s = enqueue(plan, plan->ev);
        if (s != SFT_OK) return s;
        return finish(plan, stats, true);
    }
    if (plan->stream == nullptr) {
        // the legacy default stream cannot be captured: enqueue directly
        s = enqueue(plan, nullptr);
    } else {
        if (!plan->gexec) {
            HIPCHK(hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal));
            sft_status cs = enqueue(plan, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(plan->stream, &g);
            if (cs != SFT_OK) {
                if (g) (void)hipGraphDestroy(g);
                return cs;
            }
            if (e != hipSuccess) return fail(SFT_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            plan->graph = g;
            HIPCHK(hipGraphInstantiate(&plan->gexec, plan->graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(plan->gexec, plan->stream));
    }
    if (s != SFT_OK) return s;
    if (any_sync(plan)) return finish(plan, nullptr, false);
    return SFT_OK;
}

sft_status sft_syndromes(sft_plan_t plan, const void* x_dev, void* out_dev) {
    if (!plan || !x_dev || !out_dev) return fail(SFT_E_INVALID, "plan, input or output is NULL");
    if (plan->sig.size() != 1) return fail(SFT_E_INVALID, "sft_syndromes needs a single-signal plan");
    if (plan->upload_pending) HIPCHK(hipEventSynchronize(plan->ev_upload));
    plan->h_io[0] = IoDev{x_dev, nullptr, nullptr, 0, nullptr};
    HIPCHK(hipMemcpyAsync(plan->d_io, plan->h_io, sizeof(IoDev), hipMemcpyHostToDevice, plan->stream));
    HIPCHK(hipEventRecord(plan->ev_upload, plan->stream));
    plan->upload_pending = true;
    plan->io_valid = false;
    LaunchCtx c = make_ctx(plan);
    HIPCHK(launch_zero_counters(c));
    HIPCHK(launch_syndromes(c));
    const SigHost& g = plan->sig[0];
    const size_t elems = g.mode == SFT_MODE_ITERATIVE ? 2 * (size_t)iter_bins_off(g.m, g.L) : (size_t)g.S * (size_t)g.m;
    const size_t bytes = elems * (plan->fp64 ? sizeof(double2) : sizeof(float2));
    if (g.mode == SFT_MODE_ITERATIVE)
        HIPCHK(hipMemcpyAsync(out_dev, plan->d_synd, bytes, hipMemcpyDeviceToDevice, plan->stream));
    else
        HIPCHK(launch_copy_syndromes(c, (int64_t)elems, out_dev));   // kept by bin: to [S][M]
    if (any_sync(plan)) HIPCHK(hipStreamSynchronize(plan->stream));
    return SFT_OK;
}

sft_status sft_plan_get(sft_plan_t plan, int64_t index, sft_plan_info* info) {
    if (!plan || !info) return fail(SFT_E_INVALID, "plan or info is NULL");
    if (index < 0 || index >= (int64_t)plan->sig.size()) return fail(SFT_E_INVALID, "index out of range");
    const SigHost& g = plan->sig[(size_t)index];
    std::memset(info, 0, sizeof(*info));
    info->n = g.n;
    info->k = g.k;
    info->m = g.m;
    info->d = g.d;
    info->l = g.L;
    info->r = g.R;
    info->in_dtype = g.dtype;
    info->mode = g.mode;
    info->flags = g.flags;
    info->n_signals = (int32_t)plan->sig.size();
    for (int j = 0; j < g.R; ++j) info->rshifts[j] = g.rshifts[(size_t)j];
    info->tau_zero = g.tau_zero;
    info->tau_rank = g.tau_rank;
    info->tau_res = g.tau_res;
    info->tau_amp = g.tau_amp;
    info->c_res = g.c_res;
    info->delta_grid = g.delta_grid;
    info->delta_mag = g.delta_mag;
    info->workspace_bytes = plan->ws_bytes;
    return SFT_OK;
}

void sft_destroy(sft_plan_t plan) { release(plan); }

sft_status sft_plan_attach_mlp(sft_plan_t plan, sft_mlp_t mlp) {
    if (!plan) return fail(SFT_E_INVALID, "plan is NULL");
    if (plan->gexec) {
        (void)hipGraphExecDestroy(plan->gexec);
        plan->gexec = nullptr;
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    plan->mlp = mlp;
    return SFT_OK;
}

sft_status sft_features(sft_plan_t plan, const void* x_dev, float* feat_dev, int64_t* bins_dev, int64_t capacity,
                        int64_t* count_dev) {
    if (!plan || !x_dev || !count_dev || capacity < 0 || (capacity > 0 && (!feat_dev || !bins_dev)))
        return fail(SFT_E_INVALID, "bad argument");
    if (plan->sig.size() != 1 || plan->sig[0].mode != kExact || plan->sig[0].L != 4)
        return fail(SFT_E_UNSUPPORTED, "features need a single-signal exact-mode plan with L = 4");
    if (plan->upload_pending) HIPCHK(hipEventSynchronize(plan->ev_upload));
    plan->h_io[0] = IoDev{x_dev, nullptr, nullptr, 0, nullptr};
    HIPCHK(hipMemcpyAsync(plan->d_io, plan->h_io, sizeof(IoDev), hipMemcpyHostToDevice, plan->stream));
    HIPCHK(hipEventRecord(plan->ev_upload, plan->stream));
    plan->upload_pending = true;
    plan->io_valid = false;
    LaunchCtx c = make_ctx(plan);
    HIPCHK(launch_zero_counters(c));
    HIPCHK(launch_syndromes(c));
    HIPCHK(launch_activity(c));
    sft_status s = sft_features_enqueue(c, feat_dev, bins_dev, capacity, count_dev);
    if (s != SFT_OK) return s;
    if (any_sync(plan)) HIPCHK(hipStreamSynchronize(plan->stream));
    return SFT_OK;
}

}  // extern "C"

