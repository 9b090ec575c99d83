// Step 3 of sFFT-DT on the device: per-bin syndrome decoding (Sec. II-B,
// Steps (i)-(iii), with the grid check of Alg. 1) and, for generally K-sparse
// signals, the K-vote (Sec. III-C Step 1, Alg. 2 Part 2) and the CS recovery
// of flagged bins (Steps 2-3 of pruning and Subspace Pursuit, Eq. (11)).
// One lane per bin, FP64 throughout, on de-rotated syndromes (see algebra.h).
#include "algebra.h"

namespace sft {

constexpr int kMaxR = 16;     // random shifts handled by the CS step
constexpr int kMaxCand = 8;   // pruned candidates (min(2 a, R, d) <= 8)

template <typename T>
struct V2;
template <>
struct V2<float> {
    using type = float2;
};
template <>
struct V2<double> {
    using type = double2;
};

// De-rotated syndromes of bin k: mt_l = e^{-i 2 pi (k l mod N) / N} m_l for the
// lines [line0, line0 + cnt) whose shifts are sh[0..cnt).
template <typename T, int MAXC>
__device__ inline void load_derotated(const typename V2<T>::type* __restrict__ syn, int log2m, int64_t k,
                                      int64_t n, const int64_t* sh, int cnt, zd* out) {
#pragma unroll
    for (int l = 0; l < MAXC; ++l) {
        out[l] = zd{0.0, 0.0};
        if (l < cnt) {
            auto v = syn[((int64_t)l << log2m) + k];
            zd w = unit_root((k * sh[l]) & (n - 1), n);
            out[l] = cmul_conj(w, zd{(double)v.x, (double)v.y});
        }
    }
}

__device__ inline unsigned long long sv_key(double s) {
    if (!(s >= 0.0) || !isfinite(s)) return 0ull;
    return (unsigned long long)__double_as_longlong(s);
}

// ------------------------------------------------ general mode: sigma and E_k

template <typename T>
__global__ __launch_bounds__(kBlock) void singular_values_kernel(const SigDev* __restrict__ sigs,
                                                                 const int2* __restrict__ items,
                                                                 const int64_t* __restrict__ shifts,
                                                                 const typename V2<T>::type* __restrict__ synd,
                                                                 double* __restrict__ sigma, double* __restrict__ ebin) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const SigDev& sg = sigs[it.x];
    if (sg.mode != kGeneral) return;
    const int64_t k = it.y + threadIdx.x;
    if (k >= sg.m) return;
    zd mt[2 * kMaxL];
    load_derotated<T, 2 * kMaxL>(synd + sg.synd_off, sg.log2m, k, sg.n, shifts + sg.shift_off, 2 * sg.L, mt);
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(mt[l]);   // zero beyond 2L
    double sv[kMaxL];
    hankel_singular_values(mt, sg.L, sv);
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
        if (i < sg.L) sigma[(sg.bin_off + k) * sg.L + i] = sv[i];
    ebin[sg.bin_off + k] = e;
}

// Block-wide selection of the r-th largest (0-based) 64-bit key by 8-bit
// radix digits (deterministic: only counts are accumulated).
template <typename KeyFn>
__device__ unsigned long long select_rth_largest(KeyFn key, int64_t n, int64_t r, unsigned* hist,
                                                 unsigned long long* sh_prefix, long long* sh_r) {
    unsigned long long prefix = 0ull, mask = 0ull;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            unsigned long long kv = key(i);
            if ((kv & mask) == prefix) atomicAdd(&hist[(kv >> shift) & 255ull], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            long long cum = 0;
            int dg = 255;
            for (; dg > 0; --dg) {
                if (cum + (long long)hist[dg] > r) break;
                cum += hist[dg];
            }
            r -= cum;
            prefix |= (unsigned long long)dg << shift;
            *sh_prefix = prefix;
            *sh_r = r;
        }
        __syncthreads();
        prefix = *sh_prefix;
        r = *sh_r;
        mask |= 255ull << shift;
        __syncthreads();
    }
    return prefix;
}

// One block per general-mode signal: the vote threshold (the K-th largest of
// all M L singular values, ties to the lower flat index k L + i) and the
// noise floor nu = lower median of E_k / (2L - 1/3).
__global__ __launch_bounds__(1024) void select_kernel(const SigDev* __restrict__ sigs, const int* __restrict__ gsigs,
                                                      const double* __restrict__ sigma, const double* __restrict__ ebin,
                                                      SelDev* __restrict__ sel) {
    __shared__ unsigned hist[256];
    __shared__ unsigned long long sh_prefix;
    __shared__ long long sh_r;
    __shared__ int sh_gt;
    const int s = gsigs[blockIdx.x];
    const SigDev& sg = sigs[s];
    const int64_t nv = (int64_t)sg.m * sg.L;
    const double* sgm = sigma + sg.bin_off * sg.L;
    const double* eb = ebin + sg.bin_off;
    unsigned long long thr = 0ull;
    long long thr_idx = nv;
    if ((int64_t)sg.k_votes < nv) {
        thr = select_rth_largest([&](int64_t i) { return sv_key(sgm[i]); }, nv, (int64_t)sg.k_votes - 1, hist,
                                 &sh_prefix, &sh_r);
        if (threadIdx.x == 0) sh_gt = 0;
        __syncthreads();
        int gt = 0, eq = 0;
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) {
            unsigned long long kv = sv_key(sgm[i]);
            gt += kv > thr;
        }
        atomicAdd(&sh_gt, gt);
        __syncthreads();
        const int64_t need = (int64_t)sg.k_votes - sh_gt;   // >= 1 votes among the ties
        (void)eq;
        unsigned long long idx = select_rth_largest(
            [&](int64_t i) { return sv_key(sgm[i]) == thr ? (unsigned long long)i : ~0ull; }, nv, nv - need, hist,
            &sh_prefix, &sh_r);
        thr_idx = (long long)idx;
    }
    const int64_t m = sg.m;
    unsigned long long med = select_rth_largest([&](int64_t i) { return sv_key(eb[i]); }, m, m - 1 - (m - 1) / 2,
                                                hist, &sh_prefix, &sh_r);
    if (threadIdx.x == 0) {
        SelDev o;
        o.thr_key = thr;
        o.thr_idx = thr_idx;
        o.nu = __longlong_as_double((long long)med) / (2.0 * sg.L - 1.0 / 3.0);
        o.pad = 0.0;
        sel[s] = o;
    }
}

// ------------------------------------------------------------ the decoder

struct BinOut {
    int n;                 // number of kept entries
    bool keep[kMaxL];      // entry j is kept
    int64_t t[kMaxL];
    zd p[kMaxL];
};

// One hypothesis of order a: locator, roots, grid check, least squares,
// residual judge; on acceptance drops |p_j| < tau_amp max|p|.
__device__ inline bool try_order(const zd* mt, int L, int a, double e, double nu, const SigDev& sg,
                                 const double2* tab, BinOut& o) {
    zd c[kMaxL], z[kMaxL], p[kMaxL];
    int64_t t[kMaxL];
    if (!locator(mt, a, c)) return false;
    if (!poly_roots(c, a, z)) return false;
    if (!roots_to_grid(z, a, sg.d, sg.delta_grid, sg.delta_mag, t)) return false;
    double r2;
    if (!vandermonde_ls(mt, 2 * L, t, a, sg.d, tab, sg.tab_stride, p, r2)) return false;
    if (!(r2 <= sg.tau_res2 * e + sg.c_res * (2 * L - a) * nu)) return false;
    double pmax = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j)
        if (j < a) pmax = fmax(pmax, cabs(p[j]));
    // keep |p_j| >= tau_amp max|p|, compacted in order (fixed-size moves only)
    o.n = 0;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        o.t[j] = t[j];
        o.p[j] = p[j];
    }
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) o.keep[j] = j < a && cabs(p[j]) >= sg.tau_amp * pmax;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) o.n += o.keep[j] ? 1 : 0;
    return true;
}

// Canonical order of hypotheses: a0, a0+1 .. L, then a0-1 .. 1.
__device__ inline int order_at(int a0, int L, int step) {
    return (step <= L - a0) ? a0 + step : a0 - (step - (L - a0));
}

// Least squares on the columns `sel` (positions into the candidate list)
// of Phi_{j,c} = w_d^{(t_c n_j) mod d}: coefficients and residual vector.
__device__ inline bool cs_ls(const zd* y, int R, const int64_t* nj, const int64_t* cand_t, const int* sel, int ns,
                             int64_t d, const double2* tab, int stride, zd* coef, zd* res, double& rn2) {
    zd g[kMaxCand * (kMaxCand + 1) / 2];
    for (int a = 0; a < ns; ++a) {
        int64_t ta = cand_t[sel[a]];
        zd b{0.0, 0.0};
        for (int j = 0; j < R; ++j) b = b + cmul_conj(omega(tab, stride, (ta * nj[j]) & (d - 1)), y[j]);
        coef[a] = b;
        for (int bb = 0; bb <= a; ++bb) {
            int64_t tb = cand_t[sel[bb]];
            zd s{0.0, 0.0};
            for (int j = 0; j < R; ++j)
                s = s + omega(tab, stride, (((tb - ta) * nj[j]) % d + d) & (d - 1));
            g[a * (a + 1) / 2 + bb] = s;   // sum_j conj(Phi_ja) Phi_jb
        }
    }
    if (!chol_solve<kMaxCand>(g, coef, ns)) return false;
    rn2 = 0.0;
    for (int j = 0; j < R; ++j) {
        zd e = y[j];
        for (int a = 0; a < ns; ++a) e = e - omega(tab, stride, (cand_t[sel[a]] * nj[j]) & (d - 1)) * coef[a];
        res[j] = e;
        rn2 += norm2(e);
    }
    return isfinite(rn2);
}

// Positions of the cnt largest values (ties to the lower position), sorted.
__device__ inline void top_positions(const double* v, int n, int cnt, int* out) {
    int m = 0;
    for (int i = 0; i < n; ++i) {
        // insertion into out[0..m) ordered by value desc, position asc
        if (m < cnt || v[i] > v[out[m - 1]]) {
            int pos = (m < cnt) ? m++ : cnt - 1;
            while (pos > 0 && v[i] > v[out[pos - 1]]) {
                out[pos] = out[pos - 1];
                --pos;
            }
            out[pos] = i;
        }
    }
    for (int i = 1; i < m; ++i) {   // sort positions ascending
        int x = out[i], j = i;
        while (j > 0 && out[j - 1] > x) {
            out[j] = out[j - 1];
            --j;
        }
        out[j] = x;
    }
}

// CS recovery of a flagged bin with order a0 (general mode).  Pruning Step 2:
// the min(2 a0, R, d) roots of unity with the smallest |P~(z)| (P~ from the
// order-a0 locator; a singular system leaves the bin flagged); Step 3:
// Phi_p; then Subspace Pursuit with sparsity a0 on the R random-shift
// syndromes y_j (de-rotated by e^{-i 2 pi k n_j / N}).
__device__ inline bool cs_recover(const zd* mt, const zd* y, int R, const int64_t* nj, int a0, const SigDev& sg,
                                  const double2* tab, BinOut& o) {
    const int64_t d = sg.d;
    int64_t cand[kMaxCand];
    int nc;
    zd c[kMaxL];
    if (locator(mt, a0, c)) {
        int keep = 2 * a0;
        if (keep > R) keep = R;
        if ((int64_t)keep > d) keep = (int)d;
        double best[kMaxCand];
        int64_t bt[kMaxCand];
        int m = 0;
        for (int64_t t = 0; t < d; ++t) {
            zd p, dp;
            poly_eval(c, a0, omega(tab, sg.tab_stride, t), p, dp);
            double e = norm2(p);
            if (m < keep || e < best[m - 1]) {
                int pos = (m < keep) ? m++ : keep - 1;
                while (pos > 0 && e < best[pos - 1]) {
                    best[pos] = best[pos - 1];
                    bt[pos] = bt[pos - 1];
                    --pos;
                }
                best[pos] = e;
                bt[pos] = t;
            }
        }
        nc = m;
        for (int i = 1; i < nc; ++i) {   // ascending t
            int64_t x = bt[i];
            int j = i;
            while (j > 0 && bt[j - 1] > x) {
                bt[j] = bt[j - 1];
                --j;
            }
            bt[j] = x;
        }
        for (int i = 0; i < nc; ++i) cand[i] = bt[i];
    } else {
        return false;   // singular order-a0 locator: nothing to prune with, the bin stays flagged
    }
    const int s = a0 < nc ? a0 : nc;
    double corr[kMaxCand];
    int T[kMaxL], E[kMaxL], U[2 * kMaxL], Tn[kMaxL];
    zd coef[kMaxCand], res[kMaxR], cu[kMaxCand], resn[kMaxR];
    for (int i = 0; i < nc; ++i) {
        zd b{0.0, 0.0};
        for (int j = 0; j < R; ++j) b = b + cmul_conj(omega(tab, sg.tab_stride, (cand[i] * nj[j]) & (d - 1)), y[j]);
        corr[i] = norm2(b);
    }
    top_positions(corr, nc, s, T);
    double rn2;
    if (!cs_ls(y, R, nj, cand, T, s, d, tab, sg.tab_stride, coef, res, rn2)) return false;
    for (int it = 0; it < 2 * s + 2; ++it) {
        for (int i = 0; i < nc; ++i) {
            zd b{0.0, 0.0};
            for (int j = 0; j < R; ++j)
                b = b + cmul_conj(omega(tab, sg.tab_stride, (cand[i] * nj[j]) & (d - 1)), res[j]);
            corr[i] = norm2(b);
        }
        top_positions(corr, nc, s, E);
        int nu_ = 0, ia = 0, ib = 0;   // merge sorted T and E
        while (ia < s || ib < s) {
            int v;
            if (ib >= s || (ia < s && T[ia] <= E[ib])) {
                v = T[ia++];
                if (ib < s && E[ib] == v) ++ib;
            } else {
                v = E[ib++];
            }
            U[nu_++] = v;
        }
        double dummy;
        zd rtmp[kMaxR];
        if (!cs_ls(y, R, nj, cand, U, nu_, d, tab, sg.tab_stride, cu, rtmp, dummy)) break;
        double mag[2 * kMaxL];
        for (int i = 0; i < nu_; ++i) mag[i] = norm2(cu[i]);
        int pos[kMaxL];
        top_positions(mag, nu_, s, pos);
        for (int i = 0; i < s; ++i) Tn[i] = U[pos[i]];
        zd cn[kMaxCand];
        double rn2n;
        if (!cs_ls(y, R, nj, cand, Tn, s, d, tab, sg.tab_stride, cn, resn, rn2n)) break;
        if (rn2n >= rn2) break;
        for (int i = 0; i < s; ++i) {
            T[i] = Tn[i];
            coef[i] = cn[i];
        }
        for (int j = 0; j < R; ++j) res[j] = resn[j];
        rn2 = rn2n;
    }
    o.n = s;
    for (int i = 0; i < kMaxL; ++i) {
        o.keep[i] = i < s;
        o.t[i] = i < s ? cand[T[i]] : 0;
        o.p[i] = i < s ? coef[i] : zd{0.0, 0.0};
    }
    return true;
}

__device__ inline void emit(const SigDev& sg, SigCounters* cnt, int64_t k, const BinOut& o, int64_t* st_loc,
                            double2* st_val) {
    if (o.n == 0) return;
    int pos = atomicAdd(&cnt->stage_count, o.n);
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        if (o.keep[j]) {
            if (pos < sg.stage_cap) {
                st_loc[sg.stage_off + pos] = k + o.t[j] * (int64_t)sg.m;
                st_val[sg.stage_off + pos] = double2{o.p[j].x, o.p[j].y};
            }
            ++pos;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void decode_kernel(const SigDev* __restrict__ sigs, const int2* __restrict__ items,
                                                        const int64_t* __restrict__ shifts,
                                                        const typename V2<T>::type* __restrict__ synd,
                                                        const double* __restrict__ epart,
                                                        const double* __restrict__ sigma, const SelDev* __restrict__ sel,
                                                        const double2* __restrict__ tab,
                                                        const signed char* __restrict__ orders,
                                                        SigCounters* __restrict__ cnt, int64_t* __restrict__ st_loc,
                                                        double2* __restrict__ st_val, int* __restrict__ flag_list) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    const int64_t k = it.y + threadIdx.x;
    if (k >= sg.m) return;
    const int L = sg.L;
    zd mt[2 * kMaxL];
    const int64_t* sh = shifts + sg.shift_off;
    load_derotated<T, 2 * kMaxL>(synd + sg.synd_off, sg.log2m, k, sg.n, sh, 2 * L, mt);
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(mt[l]);   // zero beyond 2L

    int a0 = 0;       // 0: rank test not yet computed
    double nu = 0.0;
    int a_pred = 0;
    if (sg.mode == kExact) {
        double eref = 0.0;
        for (int l = 0; l < 2 * L; ++l) eref += epart[sg.epart_off + l];
        eref /= (double)sg.m;
        if (!(e > sg.tau_zero2 * eref)) return;
        if (orders) a_pred = orders[sg.bin_off + k];
    } else {
        const SelDev sd = sel[s];
#pragma unroll
        for (int i = 0; i < kMaxL; ++i) {
            if (i >= L) continue;
            int64_t flat = k * L + i;
            unsigned long long kv = sv_key(sigma[(sg.bin_off + k) * L + i]);
            a0 += (kv > sd.thr_key || (kv == sd.thr_key && flat <= sd.thr_idx)) ? 1 : 0;
        }
        if (a0 == 0) return;
        nu = sd.nu;
    }
    atomicAdd(&cnt[s].active, 1);

    // Hypotheses: the learned order first (when given), then the canonical
    // order from a0 (rank test in exact mode, votes in general mode).
    BinOut o;
    o.n = 0;
    bool done = false;
    const bool has_pred = a_pred >= 1 && a_pred <= L;
    for (int step = has_pred ? -1 : 0; step < L && !done; ++step) {
        int a;
        if (step < 0) {
            a = a_pred;
        } else {
            if (a0 == 0) {
                double sv[kMaxL];
                hankel_singular_values(mt, L, sv);
                a0 = rank_order(sv, L, sg.tau_rank);
            }
            a = order_at(a0, L, step);
            if (has_pred && a == a_pred) continue;
        }
        done = try_order(mt, L, a, e, nu, sg, tab, o);
        if (step < 0 && !done) atomicAdd(&cnt[s].mlp_fb, 1);
    }
    if (!done) {
        atomicAdd(&cnt[s].flagged, 1);
        if (sg.mode == kGeneral) {
            int q = atomicAdd(&cnt[s].nflag, 1);   // q < M: each bin is queued at most once
            flag_list[sg.bin_off + q] = (int)k;
        }
        return;
    }
    emit(sg, &cnt[s], k, o, st_loc, st_val);
}

// CS step for the bins the decoder queued (general mode), one lane per bin.
template <typename T>
__global__ __launch_bounds__(kBlock) void cs_kernel(const SigDev* __restrict__ sigs, const int2* __restrict__ items,
                                                    const int64_t* __restrict__ shifts,
                                                    const typename V2<T>::type* __restrict__ synd,
                                                    const double* __restrict__ sigma, const SelDev* __restrict__ sel,
                                                    const double2* __restrict__ tab, SigCounters* __restrict__ cnt,
                                                    int64_t* __restrict__ st_loc, double2* __restrict__ st_val,
                                                    const int* __restrict__ flag_list) {
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    if (sg.mode != kGeneral) return;
    const int q = it.y + threadIdx.x;
    if (q >= cnt[s].nflag) return;
    const int64_t k = flag_list[sg.bin_off + q];
    const int L = sg.L;
    const int64_t* sh = shifts + sg.shift_off;
    zd mt[2 * kMaxL];
    load_derotated<T, 2 * kMaxL>(synd + sg.synd_off, sg.log2m, k, sg.n, sh, 2 * L, mt);
    const SelDev sd = sel[s];
    int a0 = 0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        if (i >= L) continue;
        int64_t flat = k * L + i;
        unsigned long long kv = sv_key(sigma[(sg.bin_off + k) * L + i]);
        a0 += (kv > sd.thr_key || (kv == sd.thr_key && flat <= sd.thr_idx)) ? 1 : 0;
    }
    zd y[kMaxR];
    const int R = sg.R;
    load_derotated<T, kMaxR>(synd + sg.synd_off + ((int64_t)(2 * L) << sg.log2m), sg.log2m, k, sg.n, sh + 2 * L, R, y);
    BinOut o;
    o.n = 0;
    if (!cs_recover(mt, y, R, sh + 2 * L, a0, sg, tab, o)) return;
    atomicAdd(&cnt[s].cs, 1);
    emit(sg, &cnt[s], k, o, st_loc, st_val);
}

// ------------------------------------------------------------ output lists

// keep[i] = 1 unless a general-mode signal found more than K entries, in which
// case only the K largest |values| are kept (ties to the lower location).
__global__ __launch_bounds__(kBlock) void keep_kernel(const SigDev* __restrict__ sigs, const int2* __restrict__ items,
                                                      const SigCounters* __restrict__ cnt,
                                                      const int64_t* __restrict__ st_loc,
                                                      const double2* __restrict__ st_val,
                                                      unsigned char* __restrict__ keep) {
    __shared__ double smag[kBlock];
    __shared__ int64_t sloc[kBlock];
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    int n = cnt[s].stage_count;
    if (n > sg.stage_cap) n = sg.stage_cap;
    if (it.y >= n) return;
    const int i = it.y + threadIdx.x;
    const bool valid = i < n;
    if (!(sg.mode == kGeneral && n > sg.k_votes)) {
        if (valid) keep[sg.stage_off + i] = 1;
        return;
    }
    double my = 0.0;
    int64_t myl = 0;
    if (valid) {
        double2 v = st_val[sg.stage_off + i];
        my = v.x * v.x + v.y * v.y;
        myl = st_loc[sg.stage_off + i];
    }
    int rank = 0;
    for (int base = 0; base < n; base += kBlock) {
        int j = base + threadIdx.x;
        if (j < n) {
            double2 v = st_val[sg.stage_off + j];
            smag[threadIdx.x] = v.x * v.x + v.y * v.y;
            sloc[threadIdx.x] = st_loc[sg.stage_off + j];
        }
        __syncthreads();
        int lim = n - base < kBlock ? n - base : kBlock;
        for (int q = 0; q < lim; ++q)
            rank += (smag[q] > my || (smag[q] == my && sloc[q] < myl)) ? 1 : 0;
        __syncthreads();
    }
    if (valid) keep[sg.stage_off + i] = rank < sg.k_votes ? 1 : 0;
}

// Kept entries, sorted by location (locations within a signal are distinct).
__global__ __launch_bounds__(kBlock) void sort_kernel(const SigDev* __restrict__ sigs, const IoDev* __restrict__ io,
                                                      const int2* __restrict__ items,
                                                      SigCounters* __restrict__ cnt,
                                                      const int64_t* __restrict__ st_loc,
                                                      const double2* __restrict__ st_val,
                                                      const unsigned char* __restrict__ keep) {
    __shared__ int64_t sloc[kBlock];
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    int n = cnt[s].stage_count;
    if (n > sg.stage_cap) n = sg.stage_cap;
    if (it.y > 0 && it.y >= n) return;
    const IoDev o = io[s];
    const int i = it.y + threadIdx.x;
    const bool mine = i < n && keep[sg.stage_off + i];
    const int64_t myl = mine ? st_loc[sg.stage_off + i] : 0;
    int rank = 0, kc = 0;
    for (int base = 0; base < n; base += kBlock) {
        int j = base + threadIdx.x;
        __syncthreads();
        sloc[threadIdx.x] = (j < n && keep[sg.stage_off + j]) ? st_loc[sg.stage_off + j] : INT64_MAX;
        __syncthreads();
        int lim = n - base < kBlock ? n - base : kBlock;
        for (int q = 0; q < lim; ++q) {
            rank += sloc[q] < myl ? 1 : 0;
            kc += sloc[q] != INT64_MAX ? 1 : 0;
        }
    }
    if (mine && rank < o.cap) {
        o.loc[rank] = myl;
        o.val[rank] = st_val[sg.stage_off + i];
    }
    if (it.y == 0 && threadIdx.x == 0) {
        *o.count = kc;
        cnt[s].kept = kc;
    }
}

// ------------------------------------------------------------ launchers

hipError_t launch_singular_values(const LaunchCtx& c) {
    if (!c.any_general || c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(singular_values_kernel<double>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs,
                           c.bin_items, c.shifts, (const double2*)c.synd, c.sigma, c.ebin);
    else
        hipLaunchKernelGGL(singular_values_kernel<float>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs,
                           c.bin_items, c.shifts, (const float2*)c.synd, c.sigma, c.ebin);
    return hipGetLastError();
}

hipError_t launch_select(const LaunchCtx& c) {
    if (c.n_general == 0) return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3(c.n_general), dim3(1024), 0, c.stream, c.sigs, c.general_sigs, c.sigma,
                       c.ebin, c.sel);
    return hipGetLastError();
}

hipError_t launch_output(const LaunchCtx& c) {
    if (c.n_out_items == 0) return hipSuccess;
    hipLaunchKernelGGL(keep_kernel, dim3(c.n_out_items), dim3(kBlock), 0, c.stream, c.sigs, c.out_items, c.cnt,
                       c.st_loc, c.st_val, c.keep);
    hipLaunchKernelGGL(sort_kernel, dim3(c.n_out_items), dim3(kBlock), 0, c.stream, c.sigs, c.io, c.out_items, c.cnt,
                       c.st_loc, c.st_val, c.keep);
    return hipGetLastError();
}

hipError_t launch_decode(const LaunchCtx& c) {
    if (c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(decode_kernel<double>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs, c.bin_items,
                           c.shifts, (const double2*)c.synd, c.epart, c.sigma, c.sel, c.omega, c.orders, c.cnt,
                           c.st_loc, c.st_val, c.flag_list);
    else
        hipLaunchKernelGGL(decode_kernel<float>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs, c.bin_items,
                           c.shifts, (const float2*)c.synd, c.epart, c.sigma, c.sel, c.omega, c.orders, c.cnt,
                           c.st_loc, c.st_val, c.flag_list);
    return hipGetLastError();
}

hipError_t launch_cs(const LaunchCtx& c) {
    if (!c.any_general || c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(cs_kernel<double>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs, c.bin_items,
                           c.shifts, (const double2*)c.synd, c.sigma, c.sel, c.omega, c.cnt, c.st_loc, c.st_val,
                           c.flag_list);
    else
        hipLaunchKernelGGL(cs_kernel<float>, dim3(c.n_bin_items), dim3(kBlock), 0, c.stream, c.sigs, c.bin_items,
                           c.shifts, (const float2*)c.synd, c.sigma, c.sel, c.omega, c.cnt, c.st_loc, c.st_val,
                           c.flag_list);
    return hipGetLastError();
}

}  // namespace sft
