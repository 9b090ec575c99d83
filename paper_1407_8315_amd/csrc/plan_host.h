// Host-side planning: parameter resolution, random shifts, workspace layout,
// work-item order, tables.  Pure host C++ (no device code).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"
#include "sft.h"

namespace sft {

struct SigHost {
    int64_t n = 0, k = 0, m = 0, d = 0;
    int L = 0, R = 0, S = 0, mode = 0, dtype = 0;
    uint32_t flags = 0;
    uint64_t seed = 0;
    std::vector<int64_t> rshifts;   // n_0 .. n_{R-1}
    double tau_zero = 0, tau_rank = 0, tau_res = 0, tau_amp = 0, c_res = 0, delta_grid = 0, delta_mag = 0;
};

struct PlanLayout {
    std::vector<SigDev> sigdev;           // the signals, then the views of iterative signals
    std::vector<int64_t> shifts;          // per signal: 0..2L-1, then n_j
    std::vector<double2> omega;           // e^{+2 pi i q / 2^om_log2}
    std::vector<double2> gram;            // Gram row tables of the general-mode shift sets
    std::vector<int4> synd_items;         // (sig, line0, nlines, pass 0|1); sig < 0 = padding
    std::vector<int4> synd_small_items;   // one-pass FP32 signals with M <= kFftPointsF32Small
    std::vector<int4> synd_late_items;    // general mode: the random-shift lines (read by the CS step only)
    std::vector<int4> synd_late_small_items;
    std::vector<int4> synd2_items;        // (sig, line0, nlines, 2): second FFT pass
    std::vector<int4> pair_items;         // (unit, line0, 0, 0) of pair_syndrome_kernel, by group
    int pair_off[kPairGroups] = {};
    int pair_n[kPairGroups] = {};
    std::vector<int2> line_items;         // (sig, line) of two-pass signals
    std::vector<int2> bin_items;          // (sig, bin0)
    std::vector<int2> act_items;          // (sig, bin0), tiles of kActivityTile
    std::vector<int> general_sigs;
    std::vector<int2> it_items;           // iterative mode: (sig, bin0) per iteration, concatenated
    int it_item_off[kMaxL] = {0, 0, 0, 0};
    int it_n_items[kMaxL] = {0, 0, 0, 0};
    int64_t it_st_elems = 0, it_rec_elems = 0;
    int n_iterative = 0;
    int64_t synd_elems = 0, epart_elems = 0, sigma_elems = 0, bin_elems = 0, stage_elems = 0, y_elems = 0;
    int tw_log2 = 0, om_log2 = 0;
    int n_general = 0;
};

// Largest supported downsampled length, and the largest one-pass length.
int64_t max_m(int dtype);
int64_t one_pass_m(int dtype);

// Fill defaults and validate one parameter set.
double expected_recovery(int64_t n, int64_t k, int64_t m, int l);
double model_us(int64_t n, int64_t k, int64_t m, int l, int dtype);
sft_status autotune(int64_t n, int64_t k, int dtype, double target, int64_t* m_out, int* l_out, double* rec_out,
                    double* us_out, std::string* msg);
sft_status resolve_params(const sft_params& in, bool batch, SigHost* out, std::string* msg);

// Default M for K: 4K rounded up to a power of two, at most N (Sec. II-E's
// d = N / (4K)); batch plans refine M and L with the autotuner.
int64_t default_m(int64_t n, int64_t k, int dtype);

// R distinct shifts in [0, d), uniform, from a splitmix64 stream of `seed`; ascending.
std::vector<int64_t> draw_shifts(uint64_t seed, int64_t d, int r);

void build_layout(const std::vector<SigHost>& sigs, bool fp64, PlanLayout* lay);

// The device description of one signal with every buffer offset 0 (a plan's
// layout then places it); dmax: size of the omega table the plan uses.
SigDev sigdev_of(const SigHost& g, int64_t dmax, bool fp64);

// Line pairs per block of pair_syndrome_kernel for a unit with `pairs`
// consecutive-shift line pairs of M points (FP32), or 0 when that kernel does
// not take the unit.
int pair_block(int pairs, int64_t m);

// Lines per block of the one-pass FFT of a unit of `lines` lines of M points;
// *small (nullable): the unit goes to the FP32 kernel of kFftPointsF32Small
// points per block.
int fft_lines_per_block(int64_t m, int lines, bool fp64, bool* small);

// Side streams and events that run the independent kernels of one stage (the
// orders of a round, the CS orders) as parallel branches.
struct Branching {
    hipStream_t side[kMaxL - 1];
    hipEvent_t fork;
    hipEvent_t join[kMaxL - 1];
    // general mode: the lines only the CS step reads (the random shifts) on
    // a stream of their own, from after the consecutive shifts' FFTs to just
    // before the CS step (nullptr: no such overlap)
    hipStream_t late;
    hipEvent_t late_fork, late_join;
};

// Enqueue the non-iterative path (exact and general signals) described by c on
// c.stream: syndromes, order estimate or vote, decoding rounds, CS step,
// output.  br == nullptr runs the branches of a stage in series on c.stream;
// with br and without events, general-mode plans gather and transform the
// random shifts beside the order estimate and the rounds;
// mlp != nullptr gives the exact-mode signals the learned order first; events
// (5, nullable) mark the stage boundaries.
sft_status enqueue_path(const LaunchCtx& c, const Branching* br, sft_mlp_t mlp, hipEvent_t* events);

// Record the text of a failure for sft_last_error(); returns s.
sft_status set_error(sft_status s, const std::string& msg);

void twiddle_table_f32(int log2n, std::vector<float2>* out);    // e^{-2 pi i q / 2^log2n}
void twiddle_table_f64(int log2n, std::vector<double2>* out);
void omega_table(int log2n, std::vector<double2>* out);         // e^{+2 pi i q / 2^log2n}

}  // namespace sft

// Learned mode: run the predictor over the active list, writing per-bin orders.
sft_status sft_mlp_launch_infer(sft_mlp_t mlp, const sft::LaunchCtx& c);
// Features of the active bins (training data) and their count.
sft_status sft_features_enqueue(const sft::LaunchCtx& c, float* feat, int64_t* bins, int64_t cap, int64_t* count);
