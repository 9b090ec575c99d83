// Host-side planning for the sFFT-DT device path.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>

#include "plan_host.h"

namespace sft {

static_assert(kFlagSpAll == SFT_FLAG_SP_ALL, "device copy of SFT_FLAG_SP_ALL");

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

constexpr int64_t kMaxD = int64_t(1) << 22;   // omega table bound

}  // namespace

// M up to one block's LDS runs as one FFT pass; above that, as two passes of
// M1 x M2 (each at most one block), up to 2^22.
int64_t max_m(int dtype) {
    (void)dtype;
    return int64_t(1) << 22;
}

int64_t one_pass_m(int dtype) { return dtype == SFT_C128 ? kFftPointsF64 : kFftPointsF32; }

int64_t default_m(int64_t n, int64_t k, int dtype) {
    int64_t m = 1;
    while (m < 4 * k) m <<= 1;
    if (m > n) m = n;
    int64_t cap = max_m(dtype);
    if (m > cap) m = cap;
    while (n / m > kMaxD) m <<= 1;
    return m;
}

std::vector<int64_t> draw_shifts(uint64_t seed, int64_t d, int r) {
    std::set<int64_t> got;
    uint64_t st = seed;
    while ((int)got.size() < r) {
        // unbiased draw in [0, d) for d a power of two
        int64_t v = (int64_t)(splitmix64(st) & (uint64_t)(d - 1));
        got.insert(v);
    }
    return std::vector<int64_t>(got.begin(), got.end());
}

// ---------------------------------------------------------------- autotuner

// Expected fraction of the K frequencies recovered in exact mode with
// (M, L): it is recovered when at most L - 1 of the others share its bin.
// Their number is hypergeometric: K - 1 drawn from the N - 1 other positions,
// d - 1 of which lie in the bin.
double expected_recovery(int64_t n, int64_t k, int64_t m, int l) {
    const int64_t d = n / m;
    const int64_t draws = k - 1, good = d - 1, pop = n - 1;
    auto lchoose = [](double a, double b) { return std::lgamma(a + 1.0) - std::lgamma(b + 1.0) - std::lgamma(a - b + 1.0); };
    const double ltot = lchoose((double)pop, (double)draws);
    double sum = 0.0;
    for (int64_t j = 0; j < l; ++j) {
        if (j > good || j > draws || draws - j > pop - good) continue;
        sum += std::exp(lchoose((double)good, (double)j) + lchoose((double)(pop - good), (double)(draws - j)) - ltot);
    }
    return std::min(1.0, sum);
}

// Modelled device time (microseconds) of one signal in a large batch on
// MI355X.  Gather + FFT: per line sample (2L lines of M samples), twice that
// when M needs two FFT passes through HBM, doubled again for complex128;
// decoder: per active bin (certificate, order-1 try) and per bin holding two
// or more frequencies (SVD rank test, higher orders).  The constants come from
// the exact-mode batch (N = 2^20, K = 1000, M = 4096, L = 4, 1024 signals):
// 0.39 ms for 33.5M line samples, 0.49 ms for 0.91M active bins.
constexpr double kUsPerLineSample = 1.16e-5;
constexpr double kUsPerActiveBin = 5.4e-4;
constexpr double kUsPerAliasedBin = 2.0e-3;

double model_us(int64_t n, int64_t k, int64_t m, int l, int dtype) {
    (void)n;
    double g = kUsPerLineSample * 2.0 * l * (double)m;
    if (m > one_pass_m(dtype)) g *= 2.0;
    if (dtype == SFT_C128) g *= 2.0;
    const double lam = (double)k / (double)m;
    const double active = (double)m * -std::expm1(-lam);
    const double aliased = (double)m * (1.0 - std::exp(-lam) * (1.0 + lam));
    return g + kUsPerActiveBin * active + kUsPerAliasedBin * aliased;
}

sft_status autotune(int64_t n, int64_t k, int dtype, double target, int64_t* m_out, int* l_out, double* rec_out,
                    double* us_out, std::string* msg) {
    if (n < 2 || !is_pow2(n) || n > (int64_t(1) << 40) || k < 1 || k > n || (dtype != SFT_C64 && dtype != SFT_C128) ||
        !(target >= 0.0 && target < 1.0)) {
        *msg = "autotune needs N a power of two >= 2, 1 <= K <= N, a known dtype and a target in [0, 1)";
        return SFT_E_INVALID;
    }
    if (target == 0.0) target = 0.999;
    int64_t best_m = 0, top_m = 0;
    int best_l = 0, top_l = 0;
    double best_us = 0.0, top_rec = -1.0;
    for (int l = 1; l <= kMaxL; ++l)
        for (int64_t m = 2; m <= n && m <= max_m(dtype); m <<= 1) {
            const int64_t d = n / m;
            if (d < 2 * l || d > kMaxD) continue;
            const double rec = expected_recovery(n, k, m, l), us = model_us(n, k, m, l, dtype);
            if (rec > top_rec || (rec == top_rec && us < model_us(n, k, top_m, top_l, dtype))) {
                top_rec = rec;
                top_m = m;
                top_l = l;
            }
            if (rec >= target && (best_m == 0 || us < best_us)) {
                best_us = us;
                best_m = m;
                best_l = l;
            }
        }
    if (best_m == 0) {
        if (top_m == 0) {
            *msg = "no admissible (M, L) for this N";
            return SFT_E_UNSUPPORTED;
        }
        best_m = top_m;
        best_l = top_l;
    }
    *m_out = best_m;
    *l_out = best_l;
    if (rec_out) *rec_out = expected_recovery(n, k, best_m, best_l);
    if (us_out) *us_out = model_us(n, k, best_m, best_l, dtype);
    return SFT_OK;
}

sft_status resolve_params(const sft_params& in, bool batch, SigHost* g, std::string* msg) {
    (void)batch;
    if (in.reserved != 0) {
        *msg = "reserved field must be 0";
        return SFT_E_INVALID;
    }
    if (in.in_dtype != SFT_C64 && in.in_dtype != SFT_C128) {
        *msg = "in_dtype must be SFT_C64 or SFT_C128";
        return SFT_E_INVALID;
    }
    if (in.mode != SFT_MODE_EXACT && in.mode != SFT_MODE_GENERAL && in.mode != SFT_MODE_ITERATIVE) {
        *msg = "mode must be SFT_MODE_EXACT, SFT_MODE_GENERAL or SFT_MODE_ITERATIVE";
        return SFT_E_INVALID;
    }
    if (in.n < 2 || in.k < 1 || in.k > in.n) {
        *msg = "need N >= 2 and 1 <= K <= N";
        return SFT_E_INVALID;
    }
    if (!is_pow2(in.n) || in.n > (int64_t(1) << 40)) {
        *msg = "N must be a power of two (at most 2^40)";
        return SFT_E_UNSUPPORTED;
    }
    const uint32_t known = SFT_FLAG_LEARNED | SFT_FLAG_SYNC | SFT_FLAG_CHECK_FINITE | SFT_FLAG_AUTOTUNE | SFT_FLAG_FFT64 |
                           SFT_FLAG_SP_ALL | SFT_FLAG_UNKNOWN_K;
    if (in.flags & ~known) {
        *msg = "unknown flag bits";
        return SFT_E_INVALID;
    }
    if ((in.flags & SFT_FLAG_UNKNOWN_K) &&
        (batch || in.mode != SFT_MODE_EXACT || (in.flags & (SFT_FLAG_LEARNED | SFT_FLAG_AUTOTUNE)))) {
        *msg = "SFT_FLAG_UNKNOWN_K applies to single-signal SFT_MODE_EXACT plans (not learned, not autotuned)";
        return SFT_E_INVALID;
    }
    if ((in.flags & SFT_FLAG_SP_ALL) && in.mode != SFT_MODE_GENERAL) {
        *msg = "SFT_FLAG_SP_ALL applies to SFT_MODE_GENERAL";
        return SFT_E_INVALID;
    }
    if ((in.flags & SFT_FLAG_LEARNED) && (in.mode != SFT_MODE_EXACT || !(in.l == 0 || in.l == 4))) {
        *msg = "the learned order predictor applies to SFT_MODE_EXACT with L = 4";
        return SFT_E_UNSUPPORTED;
    }
    g->n = in.n;
    g->k = in.k;
    g->dtype = in.in_dtype;
    g->mode = in.mode;
    g->flags = in.flags;
    g->seed = in.seed;
    int64_t m_in = in.m;
    int l_in = in.l;
    if (in.flags & SFT_FLAG_AUTOTUNE) {
        if (in.mode != SFT_MODE_EXACT || in.m != 0 || in.l != 0 || (in.flags & SFT_FLAG_LEARNED)) {
            *msg = "SFT_FLAG_AUTOTUNE applies to SFT_MODE_EXACT plans with m = 0 and l = 0 (not learned)";
            return SFT_E_INVALID;
        }
        sft_status st = autotune(in.n, in.k, in.in_dtype, in.target_recovery, &m_in, &l_in, nullptr, nullptr, msg);
        if (st != SFT_OK) return st;
    } else if (in.target_recovery != 0.0) {
        *msg = "target_recovery applies to SFT_FLAG_AUTOTUNE plans only";
        return SFT_E_INVALID;
    }
    g->L = l_in == 0 ? 4 : l_in;
    if (g->L < 1 || g->L > kMaxL) {
        *msg = "L must be in 1..4";
        return SFT_E_UNSUPPORTED;
    }
    if (m_in == 0 && (in.flags & SFT_FLAG_UNKNOWN_K)) m_in = std::min<int64_t>(in.n, max_m(in.in_dtype));
    g->m = m_in == 0 ? default_m(in.n, in.k, in.in_dtype) : m_in;
    if (!is_pow2(g->m) || g->m > in.n) {
        *msg = "M must be a power of two dividing N";
        return SFT_E_UNSUPPORTED;
    }
    if (g->m > max_m(in.in_dtype)) {
        *msg = "M above " + std::to_string(max_m(in.in_dtype)) + " is not supported for this input type";
        return SFT_E_UNSUPPORTED;
    }
    g->d = in.n / g->m;
    if (g->d > kMaxD) {
        *msg = "d = N/M above 2^22 is not supported";
        return SFT_E_UNSUPPORTED;
    }
    if (g->mode == SFT_MODE_ITERATIVE) {
        // iteration l runs on M_0 / 2^l bins with d_0 2^l
        if ((g->m >> (g->L - 1)) < 1) {
            *msg = "iterative mode needs M_0 >= 2^(L-1)";
            return SFT_E_UNSUPPORTED;
        }
        if ((g->d << (g->L - 1)) > kMaxD) {
            *msg = "iterative mode: d_0 2^(L-1) above 2^22 is not supported";
            return SFT_E_UNSUPPORTED;
        }
    }
    if ((int64_t)g->m * g->L > (int64_t(1) << 30)) {
        *msg = "M * L too large";
        return SFT_E_UNSUPPORTED;
    }
    if (g->mode == SFT_MODE_GENERAL) {
        int64_t r = in.r == 0 ? std::min<int64_t>(3 * g->L, g->d) : in.r;
        if (r < 1 || r > 16 || r > g->d) {
            *msg = "R must be in 1..16 and at most d";
            return SFT_E_UNSUPPORTED;
        }
        g->R = (int)r;
        g->rshifts = draw_shifts(in.seed, g->d, g->R);
        if (g->k > (int64_t)g->m * g->L) {
            *msg = "K exceeds M * L: the vote cannot assign K orders";
            return SFT_E_UNSUPPORTED;
        }
    } else {
        if (in.r != 0) {
            *msg = "R applies to SFT_MODE_GENERAL only";
            return SFT_E_INVALID;
        }
        g->R = 0;
    }
    g->S = 2 * g->L + g->R;
    const bool c128 = in.in_dtype == SFT_C128;
    auto pick = [](double v, double def) { return v == 0.0 ? def : v; };
    g->tau_zero = pick(in.tau_zero, c128 ? 1e-9 : 1e-4);
    g->tau_rank = pick(in.tau_rank, c128 ? 1e-10 : 1e-5);
    g->tau_res = pick(in.tau_res, c128 ? 1e-9 : 1e-4);
    g->tau_amp = pick(in.tau_amp, c128 ? 1e-9 : 1e-4);
    g->c_res = pick(in.c_res, 3.0);
    g->delta_grid = pick(in.delta_grid, 0.1);
    g->delta_mag = pick(in.delta_mag, 0.05);
    for (double v : {g->tau_zero, g->tau_rank, g->tau_res, g->tau_amp, g->c_res, g->delta_grid, g->delta_mag})
        if (!(v > 0.0) || !std::isfinite(v)) {
            *msg = "thresholds must be positive and finite";
            return SFT_E_INVALID;
        }
    if (g->delta_grid >= 0.5) {
        *msg = "delta_grid must be below 0.5";
        return SFT_E_INVALID;
    }
    return SFT_OK;
}

SigDev sigdev_of(const SigHost& g, int64_t dmax, bool fp64) {
    const int64_t pmax = fp64 ? kFftPointsF64 : kFftPointsF32;
    SigDev s;
    std::memset(&s, 0, sizeof(s));
    s.n = g.n;
    s.d = g.d;
    s.m = (int32_t)g.m;
    s.log2m = ilog2(g.m);
    s.L = g.L;
    s.R = g.R;
    s.S = g.S;
    s.mode = g.mode;
    s.k_votes = (int32_t)std::min<int64_t>(g.k, INT32_MAX);
    s.flags = (int32_t)g.flags;
    s.stage_cap = (int32_t)(g.m * g.L);
    s.tab_stride = (int32_t)(dmax / g.d);
    s.log2m1 = g.m > pmax ? (ilog2(g.m) + 1) / 2 : 0;   // M1 = 2^ceil(log2 M / 2)
    s.bstride = g.mode == SFT_MODE_ITERATIVE ? 0 : 2 * g.L;   // by bin (iterative grids: by line)
    s.rnd_off = (int64_t)g.m * 2 * g.L;                         // relative to synd_off; build_layout adds it
    s.view0 = -1;
    s.tau_zero2 = g.tau_zero * g.tau_zero;
    s.tau_rank = g.tau_rank;
    s.tau_res2 = g.tau_res * g.tau_res;
    s.tau_amp = g.tau_amp;
    s.c_res = g.c_res;
    s.delta_grid = g.delta_grid;
    s.delta_mag = g.delta_mag;
    return s;
}

int pair_block(int pairs, int64_t m) {
    if (pairs < 1 || m < (int64_t(1) << kPairLog2MMin) || m > (int64_t(1) << kPairLog2MMax)) return 0;
    // one pair per block where it makes whole waves (measured at M = 4096: 2
    // pairs per block are 1.35x slower, with twice the VGPRs per block), more
    // for short lines
    for (int p : {1, 2, 4}) {
        if (p > pairs || pairs % p) continue;
        const int64_t threads = p * (m >> kPairLpt);
        if (threads >= 64 && threads <= 1024) return p;
    }
    return 0;
}

int fft_lines_per_block(int64_t m, int lines, bool fp64, bool* small) {
    const bool sm = !fp64 && m <= kFftPointsF32Small;
    if (small) *small = sm;
    const int64_t pts = sm ? kFftPointsF32Small : (fp64 ? kFftPointsF64 : kFftPointsF32);
    return (int)std::max<int64_t>(1, std::min<int64_t>(lines, pts / m));
}

void build_layout(const std::vector<SigHost>& sigs, bool fp64, PlanLayout* lay) {
    const int64_t pmax = fp64 ? kFftPointsF64 : kFftPointsF32;
    int64_t mmax = 1, dmax = 1;
    for (auto& g : sigs) {
        mmax = std::max(mmax, g.m);
        dmax = std::max(dmax, g.mode == SFT_MODE_ITERATIVE ? g.d << (g.L - 1) : g.d);
    }
    lay->tw_log2 = ilog2(mmax);
    lay->om_log2 = ilog2(dmax);
    omega_table(lay->om_log2, &lay->omega);

    // CS step (general mode): the Gram matrix of the candidate columns
    // Phi_jc = w_d^{t_c n_j} has entries sum_j w_d^{(t_e - t_i) n_j}, which
    // depend on the difference t_e - t_i mod d and the shift set only:
    // F[delta] = sum_j w_d^{(delta n_j) mod d}, summed in j order from the
    // device's own omega table (one table per distinct (d, n_j) set)
    std::map<std::vector<int64_t>, int64_t> gram_of;
    auto gram_table = [&](const SigHost& g) -> int64_t {
        std::vector<int64_t> key(g.rshifts);
        key.push_back(g.d);
        auto it = gram_of.find(key);
        if (it != gram_of.end()) return it->second;
        const int64_t off = (int64_t)lay->gram.size(), stride = dmax / g.d;
        for (int64_t delta = 0; delta < g.d; ++delta) {
            double2 acc{0.0, 0.0};
            for (int64_t nj : g.rshifts) {
                const double2 w = lay->omega[(size_t)(((delta * nj) & (g.d - 1)) * stride)];
                acc.x += w.x;
                acc.y += w.y;
            }
            lay->gram.push_back(acc);
        }
        gram_of.emplace(std::move(key), off);
        return off;
    };

    // Assign signals to 8 lanes (one per XCD) by greedy balancing of their
    // syndrome work, so that every block of a signal runs on one XCD.
    const int kLanes = 8;
    std::vector<std::vector<int>> lane_sigs(kLanes);
    {
        std::vector<int> order(sigs.size());
        for (size_t i = 0; i < sigs.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return sigs[a].S * sigs[a].m > sigs[b].S * sigs[b].m;
        });
        std::vector<int64_t> load(kLanes, 0);
        for (int s : order) {
            int best = 0;
            for (int l = 1; l < kLanes; ++l)
                if (load[l] < load[best]) best = l;
            lane_sigs[best].push_back(s);
            load[best] += sigs[s].S * sigs[s].m;
        }
        for (auto& v : lane_sigs) std::sort(v.begin(), v.end());
    }

    int64_t synd = 0, ep = 0, bins = 0, stage = 0, ybuf = 0, it_st = 0, it_rec = 0;
    lay->sigdev.resize(sigs.size());
    for (size_t i = 0; i < sigs.size(); ++i) {
        const SigHost& g = sigs[i];
        SigDev& s = lay->sigdev[i];
        s = sigdev_of(g, dmax, fp64);
        s.synd_off = synd;
        s.rnd_off += synd;
        s.epart_off = ep;
        s.bin_off = bins;
        s.stage_off = stage;
        s.shift_off = (int32_t)lay->shifts.size();
        s.y_off = ybuf;
        const bool iter = g.mode == SFT_MODE_ITERATIVE;
        if (g.m > pmax && !iter) ybuf += (int64_t)g.S * g.m;
        s.parent = (int32_t)i;
        if (iter) {
            s.it_st_off = it_st;
            s.it_rec_off = it_rec;
            it_st += iter_bins_off(g.m, g.L);
            it_rec += iter_rec_off(g.m, g.L);
        }
        for (int l = 0; l < 2 * g.L; ++l) lay->shifts.push_back(l);
        for (int64_t v : g.rshifts) lay->shifts.push_back(v);
        synd += (int64_t)g.S * g.m;
        ep += g.S;
        bins += g.m;
        stage += g.m * g.L;
        if (g.mode == SFT_MODE_GENERAL) {
            lay->general_sigs.push_back((int)i);
            s.gram_off = gram_table(g);
        }
    }
    // Iterative signals: one view per iteration l, with the grid of that
    // iteration (d_0 2^l, M_0 / 2^l) and its two shifts 2l, 2l + 1, whose
    // syndromes sit after those of the earlier iterations in the signal's
    // syndrome region (2 (M_0 + M_0/2 + ...) <= 2L M_0 elements).
    for (size_t i = 0; i < sigs.size(); ++i) {
        const SigHost& g = sigs[i];
        if (g.mode != SFT_MODE_ITERATIVE) continue;
        lay->sigdev[i].view0 = (int32_t)lay->sigdev.size();
        for (int l = 0; l < g.L; ++l) {
            SigDev v = lay->sigdev[i];
            v.d = g.d << l;
            v.m = (int32_t)(g.m >> l);
            v.log2m = ilog2(v.m);
            v.S = 2;
            v.L = 1;
            v.synd_off = lay->sigdev[i].synd_off + 2 * iter_bins_off(g.m, l);
            v.epart_off = lay->sigdev[i].epart_off + 2 * l;
            v.shift_off = lay->sigdev[i].shift_off + 2 * l;
            v.tab_stride = (int32_t)(dmax / v.d);
            v.log2m1 = v.m > pmax ? (v.log2m + 1) / 2 : 0;
            v.bstride = 0;   // grids of iterative signals: by line
            v.y_off = ybuf;
            if (v.m > pmax) ybuf += 2 * (int64_t)v.m;
            v.view0 = -1;
            lay->sigdev.push_back(v);
        }
        lay->n_iterative += 1;
    }
    lay->it_st_elems = it_st;
    lay->it_rec_elems = it_rec;
    lay->synd_elems = synd;
    lay->epart_elems = ep;
    lay->bin_elems = bins;
    lay->sigma_elems = bins * kMaxL;
    lay->stage_elems = stage;
    lay->y_elems = ybuf;
    lay->n_general = (int)lay->general_sigs.size();

    // Work items per lane, then interleaved so that item id % 8 == lane: the
    // hardware hands consecutive block ids to the XCDs in turn.  Short lanes
    // are padded with no-op items.
    auto interleave = [&](auto per_signal, auto pad, auto& out) {
        using Item = typename std::decay<decltype(out)>::type::value_type;
        std::vector<std::vector<Item>> lanes(kLanes);
        for (int l = 0; l < kLanes; ++l)
            for (int s : lane_sigs[l]) per_signal(s, lanes[l]);
        size_t len = 0;
        for (auto& v : lanes) len = std::max(len, v.size());
        size_t used = 0;
        for (int l = 0; l < kLanes; ++l)
            if (!lanes[l].empty()) used = l + 1;
        if (sigs.size() < (size_t)kLanes) {
            // few signals: no padding, items of each signal stay adjacent
            for (auto& v : lanes)
                for (auto& it : v) out.push_back(it);
            return;
        }
        (void)used;
        for (size_t j = 0; j < len; ++j)
            for (int l = 0; l < kLanes; ++l) out.push_back(j < lanes[l].size() ? lanes[l][j] : pad);
    };
    // FFT units: a signal, or for an iterative signal each of its views
    // (items of one signal stay in its lane, so its views share the XCD's L2)
    auto for_units = [&](int s, auto fn) {
        const SigHost& g = sigs[s];
        if (g.mode == SFT_MODE_ITERATIVE) {
            for (int l = 0; l < g.L; ++l) {
                const int idx = lay->sigdev[s].view0 + l;
                fn(idx, (int64_t)lay->sigdev[idx].m, 2, lay->sigdev[idx].log2m1);
            }
        } else {
            fn(s, g.m, g.S, lay->sigdev[s].log2m1);
        }
    };
    // FP32 units with M <= kFftPointsF32Small: blocks of fewer points (one
    // line of 4096, or more lines of fewer) and a smaller LDS footprint, so that
    // more blocks share a CU and overlap their gathers
    const auto small = [&](int64_t m) { return !fp64 && m <= kFftPointsF32Small; };
    // Lines of a unit taken by pair_syndrome_kernel (FP32, one pass): the 2L
    // consecutive shifts of a signal, the two shifts of an iterative grid,
    // when they do not wrap around N (d > last shift); *pb = pairs per block.
    // Iterative signals whose every grid is one-pass FP32 without wrap, with
    // 2^kPairLog2MMin <= M_l and M_0 <= 2^kPairLog2MMax: all their grids in
    // one launch (iter_pair_kernel), a signal's grids in adjacent items of its
    // lane, so that the later grids' samples, which share grid 0's 128-byte
    // lines, are read from the same L2 at about the same time.
    const auto fused_iter = [&](int s) -> bool {
        const SigHost& g = sigs[(size_t)s];
        if (g.mode != SFT_MODE_ITERATIVE || fp64 || g.L < 2) return false;
        const int lm0 = ilog2(g.m);
        if (lm0 > kPairLog2MMax || lm0 - (g.L - 1) < kPairLog2MMin) return false;
        for (int l = 0; l < g.L; ++l) {
            const SigDev& u = lay->sigdev[(size_t)(lay->sigdev[(size_t)s].view0 + l)];
            if (u.log2m1 != 0 || lay->shifts[(size_t)u.shift_off] + 1 >= u.d) return false;
        }
        return true;
    };
    const auto pair_lines = [&](int idx, int* pb) -> int {
        const SigDev& u = lay->sigdev[idx];
        *pb = 0;
        if (u.mode == SFT_MODE_ITERATIVE && fused_iter(u.parent)) {
            *pb = 1;
            return 2;
        }
        if (fp64 || u.log2m1 != 0) return 0;
        const int pairs = u.mode == SFT_MODE_ITERATIVE ? 1 : u.L;
        const int64_t last = lay->shifts[(size_t)u.shift_off] + 2 * pairs - 1;
        if (last >= u.d) return 0;
        *pb = pair_block(pairs, u.m);
        return *pb ? 2 * pairs : 0;
    };
    for (int g = 0; g < kPairGroups; ++g) {
        lay->pair_off[g] = (int)lay->pair_items.size();
        interleave(
            [&](int s, std::vector<int4>& v) {
                if (fused_iter(s)) {   // one item per grid: (view, l), the signal's grids adjacent
                    if (pair_group(0, ilog2(sigs[(size_t)s].m)) == g)
                        for (int l = 0; l < sigs[(size_t)s].L; ++l)
                            v.push_back(int4{lay->sigdev[(size_t)s].view0 + l, l, 0, 0});
                    return;
                }
                for_units(s, [&](int idx, int64_t m, int S, int lm1) {
                    (void)S;
                    (void)lm1;
                    int pb = 0;
                    const int lines = pair_lines(idx, &pb);
                    if (!lines || pair_group(pb, ilog2(m)) != g) return;
                    for (int l0 = 0; l0 < lines; l0 += 2 * pb) v.push_back(int4{idx, l0, 0, 0});
                });
            },
            int4{-1, 0, 0, 0}, lay->pair_items);
        lay->pair_n[g] = (int)lay->pair_items.size() - lay->pair_off[g];
    }
    // One-pass items cover [first, S) in chunks of nl lines, cut at 2L in
    // general mode: the R random shifts (lines 2L .. S-1, read by the CS
    // step only) form the `late` lists, which the launcher may run beside
    // the order estimate and the rounds; everything else comes first.
    const auto one_pass_items = [&](int idx, int64_t m, int S, bool late, std::vector<int4>& v) {
        int pb = 0;
        const int first = pair_lines(idx, &pb);
        const bool general = lay->sigdev[idx].mode == SFT_MODE_GENERAL;
        const int cut = general ? 2 * lay->sigdev[idx].L : S;
        const int lo = late ? std::max(first, cut) : first, hi = late ? S : std::max(first, cut);
        const int nl = fft_lines_per_block(m, hi - lo, fp64, nullptr);
        for (int l0 = lo; l0 < hi; l0 += nl) v.push_back(int4{idx, l0, std::min(nl, hi - l0), 0});
    };
    for (int late = 0; late < 2; ++late) {
        interleave(
            [&](int s, std::vector<int4>& v) {
                for_units(s, [&](int idx, int64_t m, int S, int lm1) {
                    (void)lm1;
                    if (small(m)) one_pass_items(idx, m, S, late, v);
                });
            },
            int4{-1, 0, 0, 0}, late ? lay->synd_late_small_items : lay->synd_small_items);
        interleave(
            [&](int s, std::vector<int4>& v) {
                for_units(s, [&](int idx, int64_t m, int S, int lm1) {
                    if (small(m)) return;
                    if (m <= pmax) {
                        one_pass_items(idx, m, S, late, v);
                    } else if (!late) {
                        // first of two passes: S * M1 lines of length M2
                        const int lm2 = ilog2(m) - lm1;
                        const int64_t lines = (int64_t)S << lm1;
                        const int nl = (int)std::min<int64_t>(lines, pmax >> lm2);
                        for (int64_t l0 = 0; l0 < lines; l0 += nl)
                            v.push_back(int4{idx, (int)l0, (int)std::min<int64_t>(nl, lines - l0), 1});
                    }
                });
            },
            int4{-1, 0, 0, 0}, late ? lay->synd_late_items : lay->synd_items);
    }
    interleave(
        [&](int s, std::vector<int4>& v) {
            for_units(s, [&](int idx, int64_t m, int S, int lm1) {
                if (m <= pmax) return;
                // second pass: S * M2 lines of length M1
                const int lm2 = ilog2(m) - lm1;
                const int64_t lines = (int64_t)S << lm2;
                const int nl = (int)std::min<int64_t>(lines, pmax >> lm1);
                for (int64_t l0 = 0; l0 < lines; l0 += nl)
                    v.push_back(int4{idx, (int)l0, (int)std::min<int64_t>(nl, lines - l0), 2});
            });
        },
        int4{-1, 0, 0, 0}, lay->synd2_items);
    for (size_t s = 0; s < sigs.size(); ++s)
        for_units((int)s, [&](int idx, int64_t m, int S, int lm1) {
            (void)lm1;
            if (m > pmax)
                for (int l = 0; l < S; ++l) lay->line_items.push_back(int2{idx, l});
        });
    interleave(
        [&](int s, std::vector<int2>& v) {
            if (sigs[s].mode == SFT_MODE_ITERATIVE) return;
            for (int64_t b = 0; b < sigs[s].m; b += kBlock) v.push_back(int2{s, (int)b});
        },
        int2{-1, 0}, lay->bin_items);
    interleave(
        [&](int s, std::vector<int2>& v) {
            if (sigs[s].mode == SFT_MODE_ITERATIVE) return;
            for (int64_t b = 0; b < sigs[s].m; b += kActivityTile) v.push_back(int2{s, (int)b});
        },
        int2{-1, 0}, lay->act_items);
    // iterative signals: tiles of kBlock bins of the grid of each iteration
    for (int l = 0; l < kMaxL; ++l) {
        lay->it_item_off[l] = (int)lay->it_items.size();
        interleave(
            [&](int s, std::vector<int2>& v) {
                const SigHost& g = sigs[s];
                if (g.mode != SFT_MODE_ITERATIVE || l >= g.L) return;
                for (int64_t b = 0; b < (g.m >> l); b += kBlock) v.push_back(int2{s, (int)b});
            },
            int2{-1, 0}, lay->it_items);
        lay->it_n_items[l] = (int)lay->it_items.size() - lay->it_item_off[l];
    }
}

void twiddle_table_f64(int log2n, std::vector<double2>* out) {
    const int64_t n = int64_t(1) << log2n;
    out->resize((size_t)n);
    for (int64_t q = 0; q < n; ++q) {
        const double a = -2.0 * M_PI * (double)q / (double)n;
        (*out)[(size_t)q] = double2{std::cos(a), std::sin(a)};
    }
}

void twiddle_table_f32(int log2n, std::vector<float2>* out) {
    std::vector<double2> t;
    twiddle_table_f64(log2n, &t);
    out->resize(t.size());
    for (size_t i = 0; i < t.size(); ++i) (*out)[i] = float2{(float)t[i].x, (float)t[i].y};
}

void omega_table(int log2n, std::vector<double2>* out) {
    const int64_t n = int64_t(1) << log2n;
    out->resize((size_t)n);
    for (int64_t q = 0; q < n; ++q) {
        const double a = 2.0 * M_PI * (double)q / (double)n;
        (*out)[(size_t)q] = double2{std::cos(a), std::sin(a)};
    }
}

}  // namespace sft
