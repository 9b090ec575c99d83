// Iterative sFFT-DT for exactly K-sparse signals on the device (Alg. 1).
//
// Iteration l works on the grid of M_l = M_0 / 2^l bins (d_l = 2^l d_0).  The
// syndromes of its two new shifts 2l and 2l + 1 come from the FFT stage (the
// two lines of the signal's view l); those of the earlier shifts are folded
// from the finer grids they were taken on, m_{2d,j}[k] = m_{d,j}[k] +
// m_{d,j}[k + M/2] (Eq. (3): a residue class mod M/2 is the union of two
// classes mod M).  Per iteration:
//   scan   one lane per bin of the grid: SubFreq on the two new syndromes
//          (contributions of every frequency solved so far whose location is
//          k mod M_l), the activity test with T (the bins whose decode failed
//          in the previous iteration, reduced mod M_l), and at l = 0 SynDec
//          itself (a = 1: z_0 = m_1/m_0, p_0 = m_0).  For l >= 1 the active
//          bins are queued, each signal in its own region of the list (a
//          counter per signal, one atomic per block: a single list counter
//          shared by every block serialises the appends);
//   solve  (l >= 1) one block per signal, one lane per queued bin: the
//          2l + 2 syndromes folded to
//          the grid, de-rotated and reduced by SubFreq, SynDec at order
//          a = l + 1 (Steps (i)-(iii) of Sec. II-B), the grid check and the
//          exact-mode judge.
// A solved bin stores its l + 1 (location, value) pairs for the SubFreq of
// later iterations and appends them to the signal's staging list; the output
// pass sorts them as in the non-iterative mode.  What a later iteration solves
// at a location already in S is a correction (SubFreq removed the earlier
// value): it is added to the location's first staging slot, and a slot whose
// sum cancels (|sum| < tau_amp max |part|) is marked with location -1.
//
// Work is in de-rotated form: for bin k the syndrome of shift j is multiplied
// by e^{-i 2 pi k j / N}, so a frequency s = k + t M_l contributes
// p w_{d_l}^{t j}, read from the FP64 table of d-th roots.
#include "algebra.h"
#include "waves.h"

namespace sft {

template <typename T>
struct IterV;
template <>
struct IterV<float> {
    using type = float2;
};
template <>
struct IterV<double> {
    using type = double2;
};

enum : uint8_t { kIterIdle = 0, kIterSolved = 1, kIterFailed = 2 };

// SubFreq for bin k of iteration l, in de-rotated form: mt[c] (shift j0 + c,
// c < CNT) -= p w_{d_l}^{(t (j0 + c)) mod d_l} for every pair (s, p) solved in
// iterations 0 .. l-1 with s = k mod M_l, t = (s - k) / M_l.  The bins of
// iteration l' that fold into k are k + i M_l, i < 2^{l - l'}.
template <int CNT>
__device__ __attribute__((always_inline)) inline void sub_solved(zd* mt, int j0, int l, int64_t k, const SigDev& sg,
                                                                   const SigDev& v, const uint8_t* __restrict__ status,
                                                                   const int64_t* __restrict__ rs,
                                                                   const double2* __restrict__ rp,
                                                                   const double2* __restrict__ tab) {
    const int64_t m0 = sg.m;
    const int64_t dmask = v.d - 1;
#pragma unroll
    for (int lp = 0; lp < kMaxL - 1; ++lp) {
        if (lp >= l) break;
        const uint8_t* st = status + sg.it_st_off + iter_bins_off(m0, lp);
        const int64_t roff = sg.it_rec_off + iter_rec_off(m0, lp);
        const int reps = 1 << (l - lp);
#pragma unroll
        for (int i = 0; i < (1 << (kMaxL - 1)); ++i) {
            if (i >= reps) break;
            const int64_t b = k + (int64_t)i * v.m;
            if (st[b] != kIterSolved) continue;
            for (int e = 0; e <= lp; ++e) {
                const int64_t s = rs[roff + b * (lp + 1) + e];
                const double2 pv = rp[roff + b * (lp + 1) + e];
                const zd p{pv.x, pv.y};
                const int64_t t = (s - k) >> v.log2m;
#pragma unroll
                for (int c = 0; c < CNT; ++c) mt[c] = mt[c] - p * omega(tab, v.tab_stride, (t * (j0 + c)) & dmask);
            }
        }
    }
}

// Dense pass of iteration L_ over tiles of kBlock bins (one instance per
// iteration, so that the loops over the bins folding into k unroll and their
// loads issue together).  Counts and list slots are aggregated per block in
// LDS: one device atomic per block and counter.
template <typename T, int L_>
__global__ __launch_bounds__(kBlock) void iter_scan_kernel(const SigDev* __restrict__ sigs, const int2* __restrict__ items,
                                                           const typename IterV<T>::type* __restrict__ synd,
                                                           const double* __restrict__ epart,
                                                           const double2* __restrict__ tab, uint8_t* __restrict__ status,
                                                           int64_t* __restrict__ rs, double2* __restrict__ rp,
                                                           int* __restrict__ rslot,
                                                           SigCounters* __restrict__ cnt, int64_t* __restrict__ st_loc,
                                                           double2* __restrict__ st_val, int2* __restrict__ qlist,
                                                           int64_t list_cap) {
    constexpr int l = L_;
    __shared__ int n_act, n_out, base;   // active bins; solved (l = 0) or queued (l >= 1) bins; their first slot
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    const SigDev& v = sigs[sg.view0 + l];
    const int64_t k = (int64_t)it.y + threadIdx.x;
    const bool valid = k < v.m;
    const double eref = (epart[v.epart_off] + epart[v.epart_off + 1]) / (double)v.m;
    uint8_t* st = status + sg.it_st_off + iter_bins_off(sg.m, l);
    if (threadIdx.x == 0) {
        n_act = 0;
        n_out = 0;
    }
    __syncthreads();

    bool act = false, solved = false;
    zd p{0.0, 0.0};
    int64_t loc = 0;
    if (valid) {
        // the two new syndromes (shifts 2l and 2l + 1), raw: magnitudes do not
        // depend on the de-rotation, which is applied only where needed
        zd mr[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const auto x = synd[v.synd_off + (int64_t)c * v.m + k];
            mr[c] = zd{(double)x.x, (double)x.y};
        }
        if (l == 0) {
            const double e = norm2(mr[0]) + norm2(mr[1]);
            act = e > sg.tau_zero2 * eref;
            if (act) {
                // SynDec, a = 1: z_0 = m_1 / m_0, p_0 = m_0, grid check, judge
                // (de-rotated: shift 0 is unchanged, shift 1 by e^{-i 2 pi k / N})
                const zd m1 = cmul_conj(unit_root(k & (sg.n - 1), sg.n), mr[1]);
                const zd z = cdiv(m1, mr[0]);
                int64_t t[kMaxL];
                bool ok = cfinite(z) && roots_to_grid(&z, 1, v.d, sg.delta_grid, sg.delta_mag, t);
                if (ok) {
                    const zd r = m1 - mr[0] * omega(tab, v.tab_stride, t[0]);
                    ok = norm2(r) <= sg.tau_res2 * e;
                }
                if (ok) {
                    solved = true;
                    p = mr[0];
                    loc = k + t[0] * (int64_t)v.m;
                }
            }
            st[k] = !act ? kIterIdle : (solved ? kIterSolved : kIterFailed);
            if (solved) {
                rs[sg.it_rec_off + k] = loc;
                rp[sg.it_rec_off + k] = double2{p.x, p.y};
            }
        } else {
            // T: a bin of iteration l - 1 that folds into k failed
            const uint8_t* prev = status + sg.it_st_off + iter_bins_off(sg.m, l - 1);
            const bool in_t = prev[k] == kIterFailed || prev[k + v.m] == kIterFailed;
            // SubFreq changes the bin only when a bin folding into it was solved
            bool any_solved = false;
#pragma unroll
            for (int lp = 0; lp < l; ++lp) {
                const uint8_t* sp = status + sg.it_st_off + iter_bins_off(sg.m, lp);
#pragma unroll
                for (int i = 0; i < (1 << (l - lp)); ++i) any_solved |= sp[k + (int64_t)i * v.m] == kIterSolved;
            }
            double e = norm2(mr[0]) + norm2(mr[1]);
            if (any_solved) {
                zd mt[2];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    mt[c] = cmul_conj(unit_root((k * (2 * l + c)) & (sg.n - 1), sg.n), mr[c]);
                sub_solved<2>(mt, 2 * l, l, k, sg, v, status, rs, rp, tab);
                e = norm2(mt[0]) + norm2(mt[1]);
            }
            act = in_t || e > sg.tau_zero2 * eref;
            st[k] = act ? kIterFailed : kIterIdle;   // the solve pass marks the solved ones
        }
    }
    const bool out = l == 0 ? solved : act;
    int my = -1;
    if (out) my = atomicAdd(&n_out, 1);
    if (act) atomicAdd(&n_act, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (n_act) atomicAdd(&cnt[s].active, n_act);
        if (l == 0 && sg.L == 1 && n_act - n_out) atomicAdd(&cnt[s].flagged, n_act - n_out);
        if (n_out) base = atomicAdd(l == 0 ? &cnt[s].stage_count : &cnt[s].it_queued[l], n_out);
    }
    __syncthreads();
    if (out) {
        const int pos = base + my;
        if (l == 0) {
            rslot[sg.it_rec_off + k] = pos < sg.stage_cap ? pos : -1;
            if (pos < sg.stage_cap) {
                st_loc[sg.stage_off + pos] = loc;
                st_val[sg.stage_off + pos] = double2{p.x, p.y};
            }
        } else {
            // the signal's own region of list q_round(0, l): bins [bin_off, bin_off + M_0)
            qlist[(int64_t)q_round(0, l) * list_cap + sg.bin_off + pos] = int2{s, (int)k};
        }
    }
}

// SynDec at order A = l + 1 for the bins queued by the scan of iteration l:
// one block of NT threads per signal (iteration 1 queues ~10% of a signal's
// bins, iterations 2 and 3 a few: one wavefront per signal there).
template <typename T, int A, int NT>
__global__ __launch_bounds__(NT) void iter_solve_kernel(const SigDev* __restrict__ sigs,
                                                            const typename IterV<T>::type* __restrict__ synd,
                                                            const double2* __restrict__ tab,
                                                            uint8_t* __restrict__ status, int64_t* __restrict__ rs,
                                                            double2* __restrict__ rp, int* __restrict__ rslot,
                                                            SigCounters* __restrict__ cnt,
                                                            int64_t* __restrict__ st_loc, double2* __restrict__ st_val,
                                                            const int2* __restrict__ qlist, int64_t list_cap) {
    constexpr int l = A - 1;
    const int s = blockIdx.x;
    const SigDev& sg = sigs[s];
    if (sg.L <= l) return;
    const int total = cnt[s].it_queued[l];
    const int2* in = qlist + (int64_t)q_round(0, l) * list_cap + sg.bin_off;
    const SigDev& v = sigs[sg.view0 + l];
    for (int item = threadIdx.x; item < total; item += NT) {
        const int64_t k = in[item].y;
        // syndromes of shifts 0 .. 2A-1 on this grid: shift j was taken at
        // iteration j / 2 and is folded 2^{l - j/2} times
        zd mt[2 * kMaxL];
#pragma unroll
        for (int j = 0; j < 2 * kMaxL; ++j) {
            mt[j] = zd{0.0, 0.0};
            if (j >= 2 * A) continue;
            const SigDev& vj = sigs[sg.view0 + j / 2];
            const auto* row = synd + vj.synd_off + (int64_t)(j & 1) * vj.m + k;
            const int reps = 1 << (l - j / 2);
            zd acc{0.0, 0.0};
            for (int i = 0; i < reps; ++i) {
                const auto x = row[(int64_t)i * v.m];
                acc = acc + zd{(double)x.x, (double)x.y};
            }
            mt[j] = acc;
        }
        // de-rotate: shift j by e^{-i 2 pi k j / N} (running powers)
        {
            const zd w1 = unit_root(k & (sg.n - 1), sg.n);
            zd w{1.0, 0.0};
#pragma unroll
            for (int j = 0; j < 2 * A; ++j) {
                mt[j] = cmul_conj(w, mt[j]);
                w = w * w1;
            }
        }
        sub_solved<2 * A>(mt, 0, l, k, sg, v, status, rs, rp, tab);
        double e = 0.0;
#pragma unroll
        for (int j = 0; j < 2 * A; ++j) e += norm2(mt[j]);
        zd c[kMaxL], z[kMaxL], p[kMaxL];
        int64_t t[kMaxL];
        double r2 = 0.0;
        bool ok = locator(mt, A, c) && poly_roots(c, A, z) &&
                  roots_to_grid(z, A, v.d, sg.delta_grid, sg.delta_mag, t) &&
                  vandermonde_ls(mt, 2 * A, t, A, v.d, tab, v.tab_stride, p, r2) && r2 <= sg.tau_res2 * e;
        // earlier parts at the solved locations: their sum, largest part and slot
        zd tot[kMaxL];
        double big[kMaxL];
        int slot[kMaxL];
#pragma unroll
        for (int j = 0; j < kMaxL; ++j) {
            tot[j] = zd{0.0, 0.0};
            big[j] = 0.0;
            slot[j] = -1;
        }
        if (ok) {
            for (int lp = 0; lp < l; ++lp) {
                const uint8_t* st = status + sg.it_st_off + iter_bins_off(sg.m, lp);
                const int64_t roff = sg.it_rec_off + iter_rec_off(sg.m, lp);
                const int reps = 1 << (l - lp);
                for (int i = 0; i < reps; ++i) {
                    const int64_t b = k + (int64_t)i * v.m;
                    if (st[b] != kIterSolved) continue;
                    for (int e = 0; e <= lp; ++e) {
                        const int64_t idx = roff + b * (lp + 1) + e;
                        const int64_t sl = rs[idx];
#pragma unroll
                        for (int j = 0; j < A; ++j)
                            if (sl == k + t[j] * (int64_t)v.m) {
                                const double2 pv = rp[idx];
                                tot[j] = tot[j] + zd{pv.x, pv.y};
                                big[j] = fmax(big[j], cabs(zd{pv.x, pv.y}));
                                if (slot[j] < 0) slot[j] = rslot[idx];
                            }
                    }
                }
            }
        }
        int n_new = 0;
#pragma unroll
        for (int j = 0; j < A; ++j) n_new += (ok && slot[j] < 0) ? 1 : 0;
        if (l == sg.L - 1) wave_count(&cnt[s].flagged, !ok);
        int pos = wave_add(&cnt[s].stage_count, n_new);
        if (ok) {
            status[sg.it_st_off + iter_bins_off(sg.m, l) + k] = kIterSolved;
            const int64_t roff = sg.it_rec_off + iter_rec_off(sg.m, l) + k * A;
#pragma unroll
            for (int j = 0; j < A; ++j) {
                const int64_t sj = k + t[j] * (int64_t)v.m;
                int q = slot[j];
                if (q < 0) {
                    // a new location
                    q = pos < sg.stage_cap ? pos : -1;
                    ++pos;
                    if (q >= 0) {
                        st_loc[sg.stage_off + q] = sj;
                        st_val[sg.stage_off + q] = double2{p[j].x, p[j].y};
                    }
                } else {
                    // a correction of an earlier value
                    const zd sum = tot[j] + p[j];
                    const bool keep = cabs(sum) >= sg.tau_amp * fmax(big[j], cabs(p[j]));
                    st_loc[sg.stage_off + q] = keep ? sj : -1;
                    st_val[sg.stage_off + q] = double2{sum.x, sum.y};
                }
                rs[roff + j] = sj;
                rp[roff + j] = double2{p[j].x, p[j].y};
                rslot[roff + j] = q;
            }
        }
    }
}

template <typename T>
static void launch_iteration_t(const LaunchCtx& c, int l) {
    using V = typename IterV<T>::type;
    const int n = c.it_n_items[l];
    if (n == 0) return;
    auto scan = l == 0 ? iter_scan_kernel<T, 0> : l == 1 ? iter_scan_kernel<T, 1> : l == 2 ? iter_scan_kernel<T, 2>
                                                                                            : iter_scan_kernel<T, 3>;
    hipLaunchKernelGGL(scan, dim3(n), dim3(kBlock), 0, c.stream, c.sigs, c.it_items + c.it_item_off[l],
                       (const V*)c.synd, c.epart, c.omega, c.it_status, c.it_loc, c.it_val, c.it_slot, c.cnt, c.st_loc,
                       c.st_val, c.qlist, c.list_cap);
    switch (l) {
        case 1:
            hipLaunchKernelGGL((iter_solve_kernel<T, 2, 256>), dim3(c.n_sigs), dim3(256), 0, c.stream, c.sigs,
                               (const V*)c.synd, c.omega, c.it_status, c.it_loc, c.it_val, c.it_slot, c.cnt, c.st_loc,
                               c.st_val, c.qlist, c.list_cap);
            break;
        case 2:
            hipLaunchKernelGGL((iter_solve_kernel<T, 3, 64>), dim3(c.n_sigs), dim3(64), 0, c.stream, c.sigs,
                               (const V*)c.synd, c.omega, c.it_status, c.it_loc, c.it_val, c.it_slot, c.cnt, c.st_loc,
                               c.st_val, c.qlist, c.list_cap);
            break;
        case 3:
            hipLaunchKernelGGL((iter_solve_kernel<T, 4, 64>), dim3(c.n_sigs), dim3(64), 0, c.stream, c.sigs,
                               (const V*)c.synd, c.omega, c.it_status, c.it_loc, c.it_val, c.it_slot, c.cnt, c.st_loc,
                               c.st_val, c.qlist, c.list_cap);
            break;
        default:
            break;
    }
}

hipError_t launch_iteration(const LaunchCtx& c, int l) {
    if (l < 0 || l >= kMaxL) return hipErrorInvalidValue;
    if (c.fp64) launch_iteration_t<double>(c, l);
    else launch_iteration_t<float>(c, l);
    return hipGetLastError();
}

}  // namespace sft
