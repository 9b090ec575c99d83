// Step 3 of sFFT-DT on the device: per-bin syndrome decoding (Sec. II-B,
// Steps (i)-(iii), with the grid check of Alg. 1) and, for generally K-sparse
// signals, the K-vote (Sec. III-C Step 1, Alg. 2 Part 2) and the CS recovery
// of flagged bins (Steps 2-3 of pruning and Subspace Pursuit, Eq. (11)).
// One lane per bin, FP64 throughout, on de-rotated syndromes (see algebra.h).
#include "algebra.h"
#include "waves.h"

namespace sft {

constexpr int kMaxR = 16;     // random shifts handled by the CS step

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

// Raw syndromes m_l[k] of the lines [0, cnt) (cnt even, 2 <= cnt <= the
// unit's 2L consecutive shifts; no de-rotation), FP64, zero beyond cnt.  Kept
// by bin, they are one contiguous run per bin: FP32 values are read as
// 16-byte pairs.  Every load is unconditional (indices clamped to the run),
// so that they are issued together: a load behind a branch on cnt would wait
// for the one before it.
template <typename T, int MAXC>
__device__ __attribute__((always_inline)) inline void load_raw(const typename V2<T>::type* __restrict__ synd,
                                                                const SigDev& sg, int64_t k, int cnt, zd* out) {
    const typename V2<T>::type* __restrict__ run = synd + synd_at(sg, 0, k);
    if constexpr (sizeof(T) == 4) {
        const float4* __restrict__ r4 = reinterpret_cast<const float4*>(run);
        const int last = (cnt >> 1) - 1;
#pragma unroll
        for (int l = 0; l < MAXC; l += 2) {
            const float4 v = r4[min(l >> 1, last)];
            const bool on = l < cnt;
            out[l] = on ? zd{(double)v.x, (double)v.y} : zd{0.0, 0.0};
            out[l + 1] = on ? zd{(double)v.z, (double)v.w} : zd{0.0, 0.0};
        }
    } else {
#pragma unroll
        for (int l = 0; l < MAXC; ++l) {
            const auto v = run[min(l, cnt - 1)];
            out[l] = l < cnt ? zd{(double)v.x, (double)v.y} : zd{0.0, 0.0};
        }
    }
}

// The R random-shift syndromes of bin k, de-rotated on demand:
// y_j = e^{-i 2 pi (k n_j mod N) / N} m_{n_j}[k], one line at a time, so that
// a consumer can fold each y_j into its sums without holding all R of them
// in registers.
template <typename T>
struct RowSource {
    const typename V2<T>::type* __restrict__ syn;   // the bin's syndrome of the first random shift
    int log2m;                                        // the others follow M apart
    int64_t k, n;
    const int64_t* sh;                                // n_0 .. n_{R-1}
    __device__ __attribute__((always_inline)) zd at(int j) const {
        const auto v = syn[(int64_t)j << log2m];
        return cmul_conj(unit_root((k * sh[j]) & (n - 1), n), zd{(double)v.x, (double)v.y});
    }
};

// In place, for the 2L consecutive shifts l = 0 .. cnt-1:
// m_l <- e^{-i 2 pi k l / N} m_l, with the phase factors as running powers of
// e^{-i 2 pi k / N} (a few ulps after 2L - 1 products; one sincospi per bin
// instead of one per line keeps the lane's registers low).
template <int MAXC>
__device__ __attribute__((always_inline)) inline void derotate_consecutive(zd* m, int64_t k, int64_t n, int cnt) {
    const zd w1 = unit_root(k & (n - 1), n);
    zd w{1.0, 0.0};
#pragma unroll
    for (int l = 0; l < MAXC; ++l) {
        if (l < cnt) m[l] = cmul_conj(w, m[l]);
        w = w * w1;
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
    // raw syndromes: de-rotation multiplies the Hankel matrix by the same
    // unitary diagonal on both sides (e^{-i phi (i + j)} = e^{-i phi i}
    // e^{-i phi j}), which changes neither its singular values nor E_k
    zd m[2 * kMaxL];
    load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * sg.L, m);
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(m[l]);   // zero beyond 2L
    double sv[kMaxL];
    gram_singular_values(m, sg.L, sv);
#pragma unroll
    for (int i = 0; i < kMaxL; ++i)
        if (i < sg.L) sigma[(sg.bin_off + k) * sg.L + i] = sv[i];
    ebin[sg.bin_off + k] = e;
}

// ------------------------------------------------ block-wide ranking

// Ranking over n distinct keys (a, b), ascending in a, then b, by one block
// of kRankThreads threads.  Up to kRankChunk keys are sorted at once in LDS
// by a bitonic network.  block_rank() gives every key its rank (several
// chunks: sorted chunks go to scratch and each key adds, per other chunk, the
// count of that chunk's keys below it, by binary search).  Used for the
// top-K of general mode and the output order; block_radix_select() (below)
// finds single ranks: the vote threshold and the noise-floor median.
constexpr int kRankThreads = 512;
constexpr int kRankChunk = 2048;

struct RankKey {
    double a;
    long long b;
};
__device__ inline bool key_less(double a1, long long b1, double a2, long long b2) {
    return a1 < a2 || (a1 == a2 && b1 < b2);
}

struct RankLds {   // 40 KB: four blocks of kRankThreads share a CU's 160 KB
    double a[kRankChunk];
    long long b[kRankChunk];
    int idx[kRankChunk];
};

struct RankScratch {   // per-signal slices of the plan's ranking scratch
    double* a;
    long long* b;
    int* idx;
    int* rank;         // rank of key i
};

__device__ inline RankScratch rank_scratch(double* a, long long* b, int* idx, int* rank, int64_t off) {
    return RankScratch{a + off, b + off, idx + off, rank + off};
}

// Sort S[0 .. P) ascending (P a power of two; entries beyond the data padded
// with +inf keys).  Whole block; ends with a barrier.
__device__ void lds_bitonic(RankLds& S, int P) {
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int ij = i ^ j;
                if (ij > i) {
                    const bool up = (i & k) == 0;
                    const bool lo_first = key_less(S.a[i], S.b[i], S.a[ij], S.b[ij]);
                    if (up != lo_first) {
                        const double ta = S.a[i];
                        S.a[i] = S.a[ij];
                        S.a[ij] = ta;
                        const long long tb = S.b[i];
                        S.b[i] = S.b[ij];
                        S.b[ij] = tb;
                        const int ti = S.idx[i];
                        S.idx[i] = S.idx[ij];
                        S.idx[ij] = ti;
                    }
                }
            }
            __syncthreads();
        }
}

__device__ inline int pow2_at_least(int n) {
    int P = 1;
    while (P < n) P <<= 1;
    return P;
}

__device__ inline void pad_keys(RankLds& S, int from, int P) {
    for (int i = from + threadIdx.x; i < P; i += blockDim.x) {
        S.a[i] = __builtin_huge_val();
        S.b[i] = 0x7fffffffffffffffll;
        S.idx[i] = -1;
    }
}

// Sort K[0 .. P) ascending (P a power of two), single 64-bit keys.  Whole
// block; ends with a barrier.
__device__ void lds_bitonic64(unsigned long long* K, int P) {
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int ij = i ^ j;
                if (ij > i) {
                    const unsigned long long x = K[i], y = K[ij];
                    if (((i & k) == 0) == (y < x)) {
                        K[i] = y;
                        K[ij] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// g.rank[i] = position of key(i) in ascending order, i < n.  Whole block.
template <typename KeyFn>
__device__ void block_rank(KeyFn key, int n, RankLds& S, const RankScratch& g) {
    const int nch = (n + kRankChunk - 1) / kRankChunk;
    for (int c = 0; c < nch; ++c) {
        const int c0 = c * kRankChunk, cn = min(kRankChunk, n - c0);
        const int P = pow2_at_least(cn);
#pragma unroll 4
        for (int i = threadIdx.x; i < cn; i += blockDim.x) {
            const RankKey k = key(c0 + i);
            S.a[i] = k.a;
            S.b[i] = k.b;
            S.idx[i] = c0 + i;
        }
        pad_keys(S, cn, P);
        __syncthreads();
        lds_bitonic(S, P);
        for (int i = threadIdx.x; i < cn; i += blockDim.x) {
            g.rank[S.idx[i]] = i;
            if (nch > 1) {
                g.a[c0 + i] = S.a[i];
                g.b[c0 + i] = S.b[i];
                g.idx[c0 + i] = S.idx[i];
            }
        }
        __syncthreads();
    }
    if (nch == 1) return;
    // each sorted chunk in turn back in LDS; every key of the other chunks
    // adds the count of that chunk's keys below it (binary search in LDS)
    for (int c2 = 0; c2 < nch; ++c2) {
        const int c0 = c2 * kRankChunk, cn = min(kRankChunk, n - c0);
        for (int i = threadIdx.x; i < cn; i += blockDim.x) {
            S.a[i] = g.a[c0 + i];
            S.b[i] = g.b[c0 + i];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (i / kRankChunk == c2) continue;
            const double a = g.a[i];
            const long long b = g.b[i];
            int lo = 0, hi = cn;
            while (lo < hi) {   // first position whose key is not below (a, b)
                const int mid = (lo + hi) >> 1;
                if (key_less(S.a[mid], S.b[mid], a, b)) lo = mid + 1;
                else hi = mid;
            }
            g.rank[g.idx[i]] += lo;
        }
        __syncthreads();
    }
}

// LDS of block_radix_select: the keys and indices of up to CH candidates,
// the indices of the final ties, the digit histogram (kRadixCopies copies,
// lanes spread over them, so that keys of one digit contend less), the
// per-wave partials of the common-prefix pass and the broadcast scalars
// (37 KB for CH = 2048, so that four blocks of kRankThreads share a CU's
// 160 KB).
constexpr int kRadixCopies = 4;
template <int CH>
struct RadixLdsT {
    unsigned long long key[CH];
    int idx[CH];
    int tie[CH];
    int hist[kRadixCopies * 256];
    unsigned long long kor[kRankThreads / 64], kand[kRankThreads / 64];
    int sel_digit, sel_rr, sel_count, n_cand, pick;
};
using RadixLds = RadixLdsT<kRankChunk>;
// candidates the selection kernel gathers into LDS (20 KB in all: its blocks
// still fit beside four blocks of the gather + FFT kernel on one CU)
constexpr int kSelChunk = 1024;

// Index of the key of ascending rank r (0 <= r < n) in the order (ukey(i), i),
// by radix selection on the 64-bit keys, 8 bits per pass: each pass counts
// the candidates (keys matching the digits fixed so far) per next digit and
// keeps the digit that holds rank r.  A first pass finds the bits common to
// all keys (their OR and AND) and counts the keys per top byte, and the digit
// passes start at the digit of the highest bit that differs (the top byte's
// counts serve when that is the top byte).  Once the candidates fit in LDS
// they are gathered there and the remaining passes run on LDS; the passes stop
// once a single candidate is left.  Ties of the full key go to the lower
// index.  Whole block of kRankThreads; the result is the same element a full
// sort would give.
template <typename UKeyFn, int CH>
__device__ int block_radix_select(UKeyFn ukey, int n, int r, RadixLdsT<CH>& S) {
    int* hist = S.hist;
    int& sel_digit = S.sel_digit;
    int& sel_rr = S.sel_rr;
    int& n_cand = S.n_cand;
    const int lane = threadIdx.x & 63;
    int* hc = hist + (lane & (kRadixCopies - 1)) * 256;
    // bits common to all keys, and in the same pass the counts per top byte
    // (bits 56..63): when the keys differ there, that byte is the first
    // digit and its pass is already done
    for (int i = threadIdx.x; i < kRadixCopies * 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    unsigned long long kor = 0ull, kand = ~0ull;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long k = ukey(i);
        kor |= k;
        kand &= k;
        atomicAdd(&hc[(int)(k >> 56)], 1);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kor |= __shfl_xor(kor, o, 64);
        kand &= __shfl_xor(kand, o, 64);
    }
    if (lane == 0) {
        S.kor[threadIdx.x >> 6] = kor;
        S.kand[threadIdx.x >> 6] = kand;
    }
    __syncthreads();
    kor = 0ull;
    kand = ~0ull;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        kor |= S.kor[w];
        kand &= S.kand[w];
    }
    const unsigned long long diff = kor ^ kand;
    // first digit: the one holding the highest differing bit (none: all keys equal)
    const int first = diff == 0ull ? -8 : ((63 - __clzll((long long)diff)) / 8) * 8;
    unsigned long long mask = first >= 56 ? 0ull : (first < 0 ? ~0ull : ~0ull << (first + 8));
    unsigned long long prefix = kand & mask;
    int rr = r;
    bool in_lds = false;
    int nc = n;   // candidates
    for (int shift = first; shift >= 0; shift -= 8) {
        if (!in_lds && nc <= CH) {
            // gather the candidates, one LDS atomic per wave (ascending index
            // order is not kept: ties are resolved by index below)
            if (threadIdx.x == 0) n_cand = 0;
            __syncthreads();
            for (int i0 = 0; i0 < n; i0 += blockDim.x) {
                const int i = i0 + threadIdx.x;
                unsigned long long k = 0ull;
                bool take = false;
                if (i < n) {
                    k = ukey(i);
                    take = (k & mask) == prefix;
                }
                const unsigned long long bal = __ballot(take);
                if (bal != 0ull) {
                    const int leader = __ffsll((long long)bal) - 1;
                    int base = 0;
                    if (lane == leader) base = atomicAdd(&n_cand, __popcll(bal));
                    base = __shfl(base, leader, 64);
                    if (take) {
                        const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
                        S.key[pos] = k;
                        S.idx[pos] = i;
                    }
                }
            }
            __syncthreads();
            nc = n_cand;
            in_lds = true;
        }
        if (shift != 56) {   // the top byte was counted with the common bits
            for (int i = threadIdx.x; i < kRadixCopies * 256; i += blockDim.x) hist[i] = 0;
            __syncthreads();
            if (in_lds) {
                for (int j = threadIdx.x; j < nc; j += blockDim.x) {
                    const unsigned long long k = S.key[j];
                    if ((k & mask) == prefix) atomicAdd(&hc[(k >> shift) & 255], 1);
                }
            } else {
                for (int i = threadIdx.x; i < n; i += blockDim.x) {
                    const unsigned long long k = ukey(i);
                    if ((k & mask) == prefix) atomicAdd(&hc[(k >> shift) & 255], 1);
                }
            }
            __syncthreads();
        }
        if (threadIdx.x < 256) {   // fold the copies into copy 0
            int v = 0;
#pragma unroll
            for (int c = 0; c < kRadixCopies; ++c) v += hist[c * 256 + threadIdx.x];
            hist[threadIdx.x] = v;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            // wave 0: lane t holds bins 4t .. 4t+3; an inclusive scan of the
            // lane sums finds the lane, then the bin, where the count passes rr
            const int t = threadIdx.x;
            const int h0 = hist[4 * t], h1 = hist[4 * t + 1], h2 = hist[4 * t + 2], h3 = hist[4 * t + 3];
            const int own = h0 + h1 + h2 + h3;
            int inc = own;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(inc, o, 64);
                if (t >= o) inc += u;
            }
            const int exc = inc - own;
            if (exc <= rr && rr < inc) {
                int cum = exc, d = 4 * t;
                if (cum + h0 <= rr) {
                    cum += h0;
                    ++d;
                    if (cum + h1 <= rr) {
                        cum += h1;
                        ++d;
                        if (cum + h2 <= rr) {
                            cum += h2;
                            ++d;
                        }
                    }
                }
                sel_digit = d;
                sel_rr = rr - cum;
                S.sel_count = hist[d];
                if (!in_lds) n_cand = hist[d];
            } else if (t == 63 && rr >= inc) {   // not reached for 0 <= r < n: the last bin
                sel_digit = 255;
                sel_rr = rr - (inc - h3);
                S.sel_count = h3;
                if (!in_lds) n_cand = h3;
            }
        }
        __syncthreads();
        prefix |= (unsigned long long)sel_digit << shift;
        mask |= 255ull << shift;
        rr = sel_rr;
        if (!in_lds) nc = n_cand;
        const bool single = S.sel_count == 1;   // one candidate left: the lower digits decide nothing
        __syncthreads();
        if (single) break;
    }
    // the rr-th lowest index among the keys matching prefix on mask (all bits,
    // unless the digits stopped at a single candidate)
    int& pick = S.pick;
    if (threadIdx.x == 0) {
        n_cand = 0;
        pick = -1;
    }
    __syncthreads();
    if (in_lds) {
        for (int j = threadIdx.x; j < nc; j += blockDim.x)
            if ((S.key[j] & mask) == prefix) S.tie[atomicAdd(&n_cand, 1)] = S.idx[j];
        __syncthreads();
        const int ne = n_cand;
        for (int j = threadIdx.x; j < ne; j += blockDim.x) {
            const int v = S.tie[j];
            int below = 0;
            for (int t = 0; t < ne; ++t) below += S.tie[t] < v ? 1 : 0;
            if (below == rr) pick = v;
        }
    } else {
        // more than CH keys equal the selected one: count them per
        // contiguous chunk of indices, then the chunk holding rank rr finds it
        const int C = (n + blockDim.x - 1) / blockDim.x;
        const int lo = min(n, (int)threadIdx.x * C), hi = min(n, lo + C);
        int c = 0;
        for (int i = lo; i < hi; ++i) c += (ukey(i) & mask) == prefix ? 1 : 0;
        S.idx[threadIdx.x] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            int run = 0;
            for (int t = 0; t < (int)blockDim.x; ++t) {
                const int v = S.idx[t];
                S.idx[t] = run;
                run += v;
            }
        }
        __syncthreads();
        const int before = S.idx[threadIdx.x];
        if (rr >= before && rr < before + c) {
            int m = rr - before;
            for (int i = lo; i < hi; ++i)
                if ((ukey(i) & mask) == prefix) {
                    if (m == 0) {
                        pick = i;
                        break;
                    }
                    --m;
                }
        }
    }
    __syncthreads();
    const int out = pick;
    __syncthreads();
    return out;
}

// One block per general-mode signal: the vote threshold (the K-th largest of
// all M L singular values, ties to the lower flat index k L + i) and the
// noise floor nu = lower median of E_k / (2L - 1/3).
__global__ __launch_bounds__(kRankThreads) void select_kernel(const SigDev* __restrict__ sigs, const int* __restrict__ gsigs,
                                                              const double* __restrict__ sigma,
                                                              const double* __restrict__ ebin, SelDev* __restrict__ sel,
                                                              double* rk_a, long long* rk_b, int* rk_i, int* rk_r) {
    __shared__ RadixLdsT<kSelChunk> S;
    const int s = gsigs[blockIdx.x];
    const SigDev& sg = sigs[s];
    const int nv = sg.m * sg.L;
    const double* sgm = sigma + sg.bin_off * sg.L;
    const double* eb = ebin + sg.bin_off;
    (void)rk_a;
    (void)rk_b;
    (void)rk_i;
    (void)rk_r;
    unsigned long long thr = 0ull;
    long long thr_idx = nv;
    if (sg.k_votes < nv) {
        // descending singular values (non-finite ones count as 0), ties to the lower index
        // descending singular values = ascending complemented key bits
        const int i = block_radix_select([&](int i) { return ~sv_key(sgm[i]); }, nv, sg.k_votes - 1, S);
        thr = sv_key(sgm[i]);
        thr_idx = i;
    }
    // lower median of E_k
    const int im = block_radix_select([&](int i) { return sv_key(eb[i]); }, sg.m, (sg.m - 1) / 2, S);
    if (threadIdx.x == 0) {
        SelDev o;
        o.thr_key = thr;
        o.thr_idx = thr_idx;
        o.nu = __longlong_as_double((long long)sv_key(eb[im])) / (2.0 * sg.L - 1.0 / 3.0);
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

// Locator of order a and a necessary condition for its roots: |c_0| is the
// product of the root magnitudes, so when it lies outside
// [(1 - delta_mag)^a, (1 + delta_mag)^a] some root fails the grid check.
__device__ __attribute__((always_inline)) inline bool locator_check(const zd* mt, int a, const SigDev& sg, zd* c) {
    if (!locator(mt, a, c)) return false;
    double lo = 1.0, hi = 1.0;
#pragma unroll
    for (int j = 0; j < kMaxL; ++j)
        if (j < a) {
            lo *= 1.0 - sg.delta_mag;
            hi *= 1.0 + sg.delta_mag;
        }
    const double c0 = cabs(c[0]);
    return c0 >= lo && c0 <= hi;
}

// One hypothesis of order a: locator, roots, grid check, least squares,
// residual judge; on acceptance drops |p_j| < tau_amp max|p|.
__device__ __attribute__((always_inline)) inline bool try_order(const zd* mt, int L, int a, double e, double nu, const SigDev& sg,
                                 const double2* tab, BinOut& o) {
    zd c[kMaxL], z[kMaxL], p[kMaxL];
    int64_t t[kMaxL];
    if (!locator_check(mt, a, sg, c)) return false;
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
__device__ __attribute__((always_inline)) inline int order_at(int a0, int L, int step) {
    return (step <= L - a0) ? a0 + step : a0 - (step - (L - a0));
}

// Subspace Pursuit works on sets of at most KC = 2 a0 candidate columns,
// represented as bit masks so that every register array is indexed by
// unrolled constants.  Columns: Phi_{j,c} = w_d^{(t_c n_j) mod d}.  Every
// quantity SP needs follows from the candidates' Gram matrix
// G_{cc'} = sum_j conj(Phi_jc) Phi_jc', from b = Phi^H y and from ||y||^2:
// least squares on a set T solves G_T x = b_T, the residual's correlations are
// b - G x, and its energy is ||y||^2 - Re(b_T^H x).

// The candidates' Gram matrix, G_ie = F[(t_e - t_i) mod d] for any i, e (the
// signal's Gram row table F; G_ei = conj(G_ie)).  Up to 2 candidates keep
// the packed lower triangle in registers (zero rows for unused slots); with
// more, the triangle would take 2 KC (KC + 1) registers per lane, so each use
// gathers its entry from the table (a few KB, cache resident; measured faster
// for KC = 4 too, where it frees 20 registers).  Unused slots then read finite
// values, always multiplied by zero coefficients or masked.
template <int KC>
struct CandGram {
    static constexpr bool kRegs = KC <= 2;
    zd g[kRegs ? KC * (KC + 1) / 2 : 1];
    int64_t t[KC];
    const double2* f;
    int64_t dmask;
    __device__ __attribute__((always_inline)) zd at(int i, int e) const {
        if constexpr (kRegs) {
            return e <= i ? g[i * (i + 1) / 2 + e] : conj(g[e * (e + 1) / 2 + i]);
        } else {
            // a compiler barrier keeps the gather at its use: hoisted out
            // of the SP iterations, the entries would all sit in registers
            asm volatile("" ::: "memory");
            const double2 v = f[(t[e] - t[i]) & dmask];
            return zd{v.x, v.y};
        }
    }
};

// Least squares on the columns in `mask` as a fixed KC system (identity
// rows outside the mask).  Returns the residual energy in rn2.
template <int KC>
__device__ inline bool cs_ls(const CandGram<KC>& g, const zd* b, double yy, unsigned mask, zd* coef, double& rn2) {
    zd gm[KC * (KC + 1) / 2];
#pragma unroll
    for (int a = 0; a < KC; ++a) {
        const bool ia = (mask >> a) & 1u;
        coef[a] = ia ? b[a] : zd{0.0, 0.0};
#pragma unroll
        for (int bb = 0; bb <= a; ++bb) {
            const bool ib = (mask >> bb) & 1u;
            gm[a * (a + 1) / 2 + bb] = (ia && ib) ? g.at(a, bb) : (a == bb ? zd{1.0, 0.0} : zd{0.0, 0.0});
        }
    }
    if (!chol_solve<KC>(gm, coef, KC)) return false;
    double bx = 0.0;
#pragma unroll
    for (int a = 0; a < KC; ++a)
        if ((mask >> a) & 1u) bx += b[a].x * coef[a].x + b[a].y * coef[a].y;   // Re(conj(b) x)
    rn2 = fmax(yy - bx, 0.0);
    return __builtin_isfinite(rn2);
}

// |(b - G x)_c|^2 for every candidate c: correlations of the residual.
template <int KC>
__device__ inline void cs_residual_corr(const CandGram<KC>& g, const zd* b, const zd* coef, int keep, double* corr) {
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        zd r = b[c];
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            r = r - g.at(c, e) * coef[e];
        }
        corr[c] = (c < keep) ? norm2(r) : 0.0;
    }
}

// Mask of the cnt largest v[i] among i in `allowed` (ties to the lower position).
template <int KC>
__device__ inline unsigned top_mask(const double* v, unsigned allowed, int cnt) {
    unsigned out = 0u;
    for (int r = 0; r < cnt; ++r) {
        int best = -1;
        double bv = 0.0;
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            const bool ok = ((allowed >> i) & 1u) && !((out >> i) & 1u);
            if (ok && (best < 0 || v[i] > bv)) {
                best = i;
                bv = v[i];
            }
        }
        if (best < 0) break;
        out |= 1u << best;
    }
    return out;
}

// Subspace Pursuit over the first `keep` (<= KC) candidates with sparsity s;
// writes the final support mask and its coefficients.
template <int KC, typename Src>
__device__ inline bool sp_run(const int64_t* cand, int keep, unsigned all, int s, const Src& ysrc, int R,
                              const int64_t* nj, int64_t d, const double2* tab, int stride, const double2* gram,
                              unsigned& T_out, zd* coef_out) {
    // b = Phi^H y (Phi_jc = w_d^{(t_c n_j) mod d}) and ||y||^2, folding in
    // the y_j in order; G = Phi^H Phi from the signal's Gram row table:
    // G_ie = sum_j w_d^{((t_e - t_i) n_j) mod d} = F[(t_e - t_i) mod d]
    // (d a power of two: the low bits, also for a negative difference)
    //
    // Four shifts at a time: a chunk's loads (y_j, n_j, the table entries) are
    // unconditional, with indices clamped to R - 1, so that they are issued
    // together instead of each waiting behind a branch for the one before;
    // positions past R add zeros, and unused candidate slots keep b = 0.
    zd b[KC];
    CandGram<KC> g;
    double yy = 0.0;
#pragma unroll
    for (int i = 0; i < KC; ++i) b[i] = zd{0.0, 0.0};
    constexpr int kChunk = 4;
    static_assert(kMaxR % kChunk == 0, "whole chunks");
    const uint64_t qmask = (uint64_t)(d - 1);
#pragma unroll
    for (int j0 = 0; j0 < kMaxR; j0 += kChunk) {
        if (j0 < R) {
            zd yv[kChunk];
            zd wv[kChunk][KC];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const int jj = min(j0 + c, R - 1);
                const uint64_t nv = (uint64_t)nj[jj];
                yv[c] = ysrc.at(jj);
#pragma unroll
                for (int i = 0; i < KC; ++i) wv[c][i] = omega(tab, stride, (int64_t)(((uint64_t)cand[i] * nv) & qmask));
            }
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const zd yj = (j0 + c < R) ? yv[c] : zd{0.0, 0.0};
                yy += norm2(yj);
#pragma unroll
                for (int i = 0; i < KC; ++i)
                    if (i < keep) b[i] = b[i] + cmul_conj(wv[c][i], yj);
            }
        }
    }
    g.f = gram;
    g.dmask = d - 1;
#pragma unroll
    for (int i = 0; i < KC; ++i) g.t[i] = cand[i];
    if constexpr (CandGram<KC>::kRegs) {
#pragma unroll
        for (int i = 0; i < KC; ++i)
#pragma unroll
            for (int e = 0; e <= i; ++e) {
                // unconditional load (unused slots hold INT64_MAX: any index
                // mod d is in range), then zero rows for unused slots
                const double2 f = gram[(cand[e] - cand[i]) & (d - 1)];
                g.g[i * (i + 1) / 2 + e] = i < keep ? zd{f.x, f.y} : zd{0.0, 0.0};
            }
    }
    double corr[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) corr[i] = norm2(b[i]);
    unsigned T = top_mask<KC>(corr, all, s);
    zd coef[KC];
    double rn2;
    if (!cs_ls<KC>(g, b, yy, T, coef, rn2)) return false;
    for (int it = 0; it < 2 * s + 2; ++it) {
        cs_residual_corr<KC>(g, b, coef, keep, corr);
        const unsigned U = T | top_mask<KC>(corr, all, s);
        // U = T: least squares on U is that on T, whose s columns are then
        // kept: no change, so the iteration would stop (exact shortcut)
        if (U == T) break;
        zd cu[KC];
        double dummy;
        if (!cs_ls<KC>(g, b, yy, U, cu, dummy)) break;
        double mag[KC];
#pragma unroll
        for (int i = 0; i < KC; ++i) mag[i] = norm2(cu[i]);
        const unsigned Tn = top_mask<KC>(mag, U, s);
        if (Tn == T) break;   // the same residual as the current one: stop (exact shortcut)
        zd cn[KC];
        double rn2n;
        if (!cs_ls<KC>(g, b, yy, Tn, cn, rn2n)) break;
        if (rn2n >= rn2) break;
        T = Tn;
        rn2 = rn2n;
#pragma unroll
        for (int i = 0; i < KC; ++i) coef[i] = cn[i];
    }
    T_out = T;
#pragma unroll
    for (int i = 0; i < KC; ++i) coef_out[i] = coef[i];
    return true;
}

// CS recovery of a flagged bin with order a0 (general mode).  Pruning Step 2:
// the min(2 a0, R, d) roots of unity with the smallest |P~(z)| (P~ from the
// order-a0 locator; a singular system leaves the bin flagged); Step 3:
// Phi_p; then Subspace Pursuit with sparsity a0 on the R random-shift
// syndromes y_j (de-rotated by e^{-i 2 pi k n_j / N}): start from the a0
// columns most correlated with y, then repeatedly merge the a0 columns most
// correlated with the residual, solve least squares on the merged set, keep
// its a0 largest coefficients, re-solve, and stop once the residual stops
// decreasing.
//
// G > 1: the bin is handled by a group of G adjacent lanes (all with the same
// inputs), which split the scan over the d roots of unity; every later step
// runs in all G lanes alike.
template <int A0, int G, typename Src>
__device__ inline bool cs_recover(const zd* mt, const Src& ysrc, int R, const int64_t* nj, const SigDev& sg,
                                  const double2* tab, const double2* gram, BinOut& o) {
    const int a0 = A0;
    constexpr int KC = 2 * A0;   // candidate bound min(2 a0, R, d) <= 2 A0
    const int64_t d = sg.d;
    zd c[kMaxL];
    if (!locator(mt, a0, c)) return false;   // nothing to prune with: the bin stays flagged
    int keep = 2 * a0;
    if (keep > R) keep = R;
    if ((int64_t)keep > d) keep = (int)d;
    // the `keep` smallest |P~(w_d^t)|, ties to the lower t (kept sorted by error)
    double best[KC];
    int64_t bt[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) {
        best[i] = __builtin_inf();
        bt[i] = INT64_MAX;
    }
    if constexpr (A0 == 1) {
        // P~(z) = z + c_0: on the unit circle |z + c_0|^2 = 1 + |c_0|^2 - 2 |c_0| cos(angle
        // between z and -c_0), increasing with the angular distance to -c_0, so the
        // smallest values sit at the grid points bracketing that angle (an exact
        // grid angle leaves two equidistant neighbours: the lower t goes first)
        const double u0 = atan2(-c[0].y, -c[0].x) * ((double)d / (2.0 * M_PI));
        double u = u0 < 0.0 ? u0 + (double)d : u0;
        int64_t t1 = (int64_t)floor(u);
        if (t1 >= d) t1 -= d;
        const double f = u - floor(u);
        const int64_t up = (t1 + 1) & (d - 1), dn = (t1 + d - 1) & (d - 1);   // d a power of two
        int64_t first = t1, second = up;
        if (f > 0.5) {
            first = up;
            second = t1;
        } else if (f == 0.5) {
            first = t1 < up ? t1 : up;
            second = t1 < up ? up : t1;
        } else if (f == 0.0 && d > 2) {
            second = dn < up ? dn : up;
        }
        if (c[0].x == 0.0 && c[0].y == 0.0) {   // |P~| = 1 everywhere: the lowest t's
            first = 0;
            second = 1 & (d - 1);
        }
        bt[0] = first;
        if (keep > 1) bt[1] = second;
    } else if constexpr (G > 1) {
        // lane gl of the group scans t = gl, gl + G, ... (w_d^t from the
        // table) into its own sorted list of the `keep` smallest |P~|^2, ties
        // to the lower t; then `keep` rounds take the smallest head over the
        // group, (e, t) in lexicographic order, and its lane pops it: the same
        // set as one scan over all t with the same values
        const int gl = threadIdx.x & (G - 1);
        double worst = __builtin_inf();   // best[keep - 1], refreshed after each insertion
        for (int64_t t = gl; t < d; t += G) {
            const zd z = omega(tab, sg.tab_stride, t);
            zd p, dp;
            poly_eval(c, a0, z, p, dp);
            const double e = norm2(p);
            if (!(e < worst)) continue;
            double ce = e;
            int64_t ct = t;
#pragma unroll
            for (int i = 0; i < KC; ++i) {
                if (i < keep && ce < best[i]) {
                    double te = best[i];
                    int64_t tt = bt[i];
                    best[i] = ce;
                    bt[i] = ct;
                    ce = te;
                    ct = tt;
                }
            }
#pragma unroll
            for (int i = 0; i < KC; ++i)
                if (i == keep - 1) worst = best[i];
        }
        int64_t sel[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            sel[r] = INT64_MAX;
            if (r < keep) {   // the same in every lane of the group
                double me = best[0];
                long long mtt = bt[0];
#pragma unroll
                for (int off = G / 2; off > 0; off >>= 1) {
                    const double oe = __shfl_xor(me, off);
                    const long long ot = __shfl_xor(mtt, off);
                    if (oe < me || (oe == me && ot < mtt)) {
                        me = oe;
                        mtt = ot;
                    }
                }
                sel[r] = mtt;
                if (bt[0] == mtt) {   // this lane's head was taken
#pragma unroll
                    for (int i = 0; i < KC - 1; ++i) {
                        best[i] = best[i + 1];
                        bt[i] = bt[i + 1];
                    }
                    best[KC - 1] = __builtin_inf();
                    bt[KC - 1] = INT64_MAX;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) bt[r] = sel[r];
    } else {
    // running powers of w_d, refreshed from the table every 64 steps
    const zd w1 = omega(tab, sg.tab_stride, 1 & (d - 1));
    zd z{1.0, 0.0};
    double worst = __builtin_inf();   // best[keep - 1], refreshed after each insertion
    for (int64_t t = 0; t < d; ++t) {
        if ((t & 63) == 0) z = omega(tab, sg.tab_stride, t);
        zd p, dp;
        poly_eval(c, a0, z, p, dp);
        z = z * w1;
        double e = norm2(p);
        if (!(e < worst)) continue;
        // insertion into the sorted prefix of length keep (fixed-index shifts)
        double ce = e;
        int64_t ct = t;
#pragma unroll
        for (int i = 0; i < KC; ++i) {
            if (i < keep && ce < best[i]) {
                double te = best[i];
                int64_t tt = bt[i];
                best[i] = ce;
                bt[i] = ct;
                ce = te;
                ct = tt;
            }
        }
#pragma unroll
        for (int i = 0; i < KC; ++i)
            if (i == keep - 1) worst = best[i];
    }
    }
    // candidates in ascending t (positions 0..keep-1), unused slots last
    int64_t cand[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) cand[i] = bt[i];
#pragma unroll
    for (int i = 0; i < KC; ++i)
#pragma unroll
        for (int j = 0; j < KC - 1; ++j)
            if (cand[j] > cand[j + 1]) {
                int64_t x = cand[j];
                cand[j] = cand[j + 1];
                cand[j + 1] = x;
            }
    const unsigned all = (1u << keep) - 1u;
    const int s = a0 < keep ? a0 : keep;
    unsigned T = 0u;
    zd coef[KC];
    bool ok;
    ok = sp_run<KC>(cand, keep, all, s, ysrc, R, nj, d, tab, sg.tab_stride, gram + sg.gram_off, T, coef);
    if (!ok) return false;
    // emit the members of T in ascending t
    o.n = 0;
    int q = 0;
#pragma unroll
    for (int i = 0; i < kMaxL; ++i) {
        o.keep[i] = false;
        o.t[i] = 0;
        o.p[i] = zd{0.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < KC; ++i) {
        if ((T >> i) & 1u) {
#pragma unroll
            for (int j = 0; j < kMaxL; ++j)
                if (j == q) {
                    o.keep[j] = true;
                    o.t[j] = cand[i];
                    o.p[j] = coef[i];
                }
            ++q;
        }
    }
    o.n = q;
    return true;
}

// Append the kept entries of a bin to its signal's staging list.  Every
// running lane of the wave calls this (with o.n = 0 when it has nothing).
__device__ __attribute__((always_inline)) inline void emit(const SigDev& sg, SigCounters* cnt, int64_t k, const BinOut& o, int64_t* st_loc,
                            double2* st_val) {
    int pos = wave_add(&cnt->stage_count, o.n);
#pragma unroll
    for (int j = 0; j < kMaxL; ++j) {
        if (o.n > 0 && o.keep[j]) {
            if (pos < sg.stage_cap) {
                st_loc[sg.stage_off + pos] = k + o.t[j] * (int64_t)sg.m;
                st_val[sg.stage_off + pos] = double2{o.p[j].x, o.p[j].y};
            }
            ++pos;
        }
    }
}

// ------------------------------------------------------------ work queues

// Order sequence of a bin: the learned order ap first (when given), then the
// canonical order from a0 without ap.  Returns the i-th order (i < L).
__device__ __attribute__((always_inline)) inline int seq_order(int a0, int ap, int L, int i) {
    if (ap < 1) return order_at(a0, L, i);
    if (i == 0) return ap;
    int n = 0, a = 0;
#pragma unroll
    for (int st = 0; st < kMaxL; ++st) {
        if (st >= L) break;
        const int b = order_at(a0, L, st);
        if (b == ap) continue;
        if (n == i - 1 && a == 0) a = b;
        ++n;
    }
    return a;
}

// Activity pass: exact mode tests E_k > tau_zero^2 mean E and lists the bin
// in the active list; general mode counts the bin's votes a0 and queues it for
// round 0 at order a0.  One block per tile of up to kActivityTile bins of a
// signal stages its bins in LDS and reserves room with one atomic per queue.
__global__ __launch_bounds__(kBlock) void activity_kernel(const SigDev* __restrict__ sigs,
                                                          const int2* __restrict__ items,
                                                          const float2* __restrict__ synd32,
                                                          const double2* __restrict__ synd64,
                                                          const double* __restrict__ epart,
                                                          const double* __restrict__ sigma,
                                                          const SelDev* __restrict__ sel,
                                                          WorkCounters* __restrict__ work, int2* __restrict__ active,
                                                          int2* __restrict__ qlist, int64_t list_cap,
                                                          SigCounters* __restrict__ cnt) {
    __shared__ int st_code[kActivityTile];
    __shared__ int st_qs[kActivityTile];   // queue << 16 | slot within the queue
    __shared__ int n_here;
    __shared__ BlockQueues bq;
    const int2 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x;
    const SigDev& sg = sigs[s];
    const int L = sg.L;
    const int64_t k0 = it.y;
    const int64_t k1 = (k0 + kActivityTile < sg.m) ? k0 + kActivityTile : sg.m;
    if (threadIdx.x == 0) n_here = 0;
    bq.reset();
    double eref = 0.0;
    for (int l = 0; l < 2 * L; ++l) eref += epart[sg.epart_off + l];
    eref /= (double)sg.m;
    SelDev sd{};
    if (sg.mode != kExact) sd = sel[s];
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kBlock) {
        int a0 = 0;
        bool act;
        if (sg.mode == kExact) {
            // the bin's 2L syndromes as one run of unconditional loads
            zd mr[2 * kMaxL];
            if (synd32)
                load_raw<float, 2 * kMaxL>(synd32, sg, k, 2 * L, mr);
            else
                load_raw<double, 2 * kMaxL>(synd64, sg, k, 2 * L, mr);
            double e = 0.0;
#pragma unroll
            for (int l = 0; l < 2 * kMaxL; ++l) e += mr[l].x * mr[l].x + mr[l].y * mr[l].y;   // zero beyond 2L
            act = e > sg.tau_zero2 * eref;
        } else {
            // the bin's L singular values, loaded unconditionally (index
            // clamped to the bin's run), counted for i < L
            const double* sb = sigma + (sg.bin_off + k) * L;
            double sv[kMaxL];
#pragma unroll
            for (int i = 0; i < kMaxL; ++i) sv[i] = sb[min(i, L - 1)];
#pragma unroll
            for (int i = 0; i < kMaxL; ++i) {
                const int64_t flat = k * L + i;
                const unsigned long long kv = sv_key(sv[i]);
                a0 += (i < L && (kv > sd.thr_key || (kv == sd.thr_key && flat <= sd.thr_idx))) ? 1 : 0;
            }
            act = a0 > 0;
        }
        if (act) {
            // general mode with every voted bin to CS (Alg. 2 as printed): CS queue entries are (signal, k)
            const bool sp_all = sg.mode != kExact && (sg.flags & kFlagSpAll);
            const int q = sg.mode == kExact ? kQueues : (sp_all ? q_cs(a0) : q_round(0, a0));
            const int pos = atomicAdd(&n_here, 1);
            st_code[pos] = sp_all ? (int)k : pack_code(k, 0, 0, a0);
            st_qs[pos] = (q << 16) | bq.reserve(q);
        }
    }
    __syncthreads();
    if (threadIdx.x <= kQueues && bq.cnt[threadIdx.x] > 0)
        bq.base[threadIdx.x] = atomicAdd(queue_counter(work, threadIdx.x), bq.cnt[threadIdx.x]);
    if (threadIdx.x == 0) atomicAdd(&cnt[s].active, n_here);
    __syncthreads();
    for (int i = threadIdx.x; i < n_here; i += kBlock) {
        const int q = st_qs[i] >> 16, slot = st_qs[i] & 0xffff;
        queue_list(active, qlist, list_cap, q)[bq.base[q] + slot] = int2{s, st_code[i]};
    }
}

// Rank test of exact-mode bins (the exact-case analogue of Pruning Step 1):
// a0 = #{sigma_i > tau_rank sigma_1} of the L x L Hankel matrix.
//
// Certificate pass, over the active list: a bin the rank-one certificate
// settles (a0 = 1, so order 1 comes first) is tried at order 1 at once:
// emitted, or queued for round 1 at its next order.  The other bins are
// queued as pending: every lane of this pass runs the same short code.
template <typename T>
__global__ __launch_bounds__(kBlock) void certify_kernel(const SigDev* __restrict__ sigs,
                                                         const typename V2<T>::type* __restrict__ synd,
                                                         const double2* __restrict__ tab, SigCounters* __restrict__ cnt,
                                                         int64_t* __restrict__ st_loc, double2* __restrict__ st_val,
                                                         WorkCounters* __restrict__ work, int2* __restrict__ active,
                                                         int2* __restrict__ qlist, int64_t list_cap) {
    __shared__ BlockQueues bq;
    const int total = work->n_active;
    for (int base0 = blockIdx.x * kBlock; base0 < total; base0 += gridDim.x * kBlock) {
        bq.reset();
        const int item = base0 + threadIdx.x;
        int q = -1;
        int2 ent{0, 0};
        if (item < total) {
            const int2 en = active[item];
            const int s = en.x;
            const int64_t k = code_k(en.y);
            // by value: the fields are read together, not at their first use behind a branch
            const SigDev sg = sigs[s];
            const int L = sg.L;
            zd mt[2 * kMaxL];
            load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
            double e = 0.0;
#pragma unroll
            for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(mt[l]);   // zero beyond 2L
            derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
            if (rank_one_certified(mt, L, sg.tau_rank)) {
                BinOut o;
                o.n = 0;
                if (try_order(mt, L, 1, e, 0.0, sg, tab, o)) {
                    emit(sg, &cnt[s], k, o, st_loc, st_val);
                } else if (L > 1) {
                    q = q_round(1, order_at(1, L, 1));
                    ent = int2{s, pack_code(k, 1, 0, 1)};
                } else {
                    wave_count(&cnt[s].flagged, true);
                }
            } else {
                q = kQPending;
                ent = int2{s, pack_code(k, 0, 0, 0)};
            }
        }
        const int slot = bq.reserve(q);
        bq.commit(work, active, qlist, list_cap, q, slot, ent);
    }
}

// SVD pass: a0 from the Jacobi singular values, for the bins of queue q_in;
// each bin goes to set `set_out` at the order of its current step (the
// learned order, when given, stays first in its sequence).
template <typename T>
__global__ __launch_bounds__(kBlock) void svd_rank_kernel(const SigDev* __restrict__ sigs,
                                                          const typename V2<T>::type* __restrict__ synd,
                                                          WorkCounters* __restrict__ work, int2* __restrict__ active,
                                                          int2* __restrict__ qlist, int64_t list_cap, int q_in,
                                                          int set_out) {
    __shared__ BlockQueues bq;
    const int total = work->q[q_in];
    const int2* in = qlist + (int64_t)q_in * list_cap;
    for (int base0 = blockIdx.x * kBlock; base0 < total; base0 += gridDim.x * kBlock) {
        bq.reset();
        const int item = base0 + threadIdx.x;
        int q = -1;
        int2 ent{0, 0};
        if (item < total) {
            const int2 en = in[item];
            const int s = en.x;
            const int code = en.y;
            const int64_t k = code_k(code);
            const int step = code_step(code), ap = code_ap(code);
            // by value: the fields are read together, not at their first use behind a branch
            const SigDev sg = sigs[s];
            const int L = sg.L;
            zd mt[2 * kMaxL];
            load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
            derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
            double sv[kMaxL];
            hankel_singular_values(mt, L, sv);
            const int a0 = rank_order(sv, L, sg.tau_rank);
            q = q_round(set_out, seq_order(a0, ap, L, step));
            ent = int2{s, pack_code(k, step, ap, a0)};
        }
        const int slot = bq.reserve(q);
        bq.commit(work, active, qlist, list_cap, q, slot, ent);
    }
}

// One round of the decoder for the bins whose next hypothesis has order A
// (round r reads set r % 2): locator, roots, grid check, least squares and
// judge for that order only.  Accepted bins are emitted; rejected ones move
// to the next round at their next order (or to the rank test, for a bin whose
// learned order failed), and a bin with no order left is flagged: counted,
// and in general mode queued for the CS step by its vote order.
// (orders 1-2: held to three waves per SIMD, measured faster than two waves
// without the order-1 kernel's few spilled registers)
template <typename T, int A, int PHASE>
__global__ __launch_bounds__(kBlock, A <= 2 ? 3 : 2) void round_kernel(const SigDev* __restrict__ sigs, const int64_t* __restrict__ shifts,
                                                       const typename V2<T>::type* __restrict__ synd,
                                                       const SelDev* __restrict__ sel, const double2* __restrict__ tab,
                                                       SigCounters* __restrict__ cnt, int64_t* __restrict__ st_loc,
                                                       double2* __restrict__ st_val, WorkCounters* __restrict__ work,
                                                       int2* __restrict__ active, int2* __restrict__ qlist,
                                                       int64_t list_cap, int round, unsigned char* __restrict__ prechk) {
    __shared__ BlockQueues bq;
    const int set_in = round & 1;
    const int q_in = PHASE == 2 ? q_roots(set_in, A) : q_round(set_in, A);
    const int total = work->q[q_in];
    const int2* in = qlist + (int64_t)q_in * list_cap;
    for (int base0 = blockIdx.x * kBlock; base0 < total; base0 += gridDim.x * kBlock) {
        bq.reset();
        const int item = base0 + threadIdx.x;
        int q = -1;
        int2 ent{0, 0};
        if (item < total) {
            const int2 en = in[item];
            const int s = en.x;
            const int code = en.y;
            const int64_t k = code_k(code);
            const int step = code_step(code), ap = code_ap(code), a0 = code_a0(code);
            // by value: the fields are read together, not at their first use
            // behind a branch (as in rest_kernel, which decodes the same
            // hypotheses when a plan has no general-mode signal: the two must
            // compile try_order alike for a batch to equal single calls bit
            // for bit; by reference here, the values differ in the last bits)
            const SigDev sg = sigs[s];
            const int L = sg.L;
            const bool exact = sg.mode == kExact;
            zd mt[2 * kMaxL];
            load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
            double e = 0.0;
#pragma unroll
            for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(mt[l]);
            derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
            const double nu = exact ? 0.0 : sel[s].nu;
            BinOut o;
            o.n = 0;
            zd cpre[kMaxL];
            if (PHASE == 1 && locator_check(mt, A, sg, cpre)) {
                q = q_roots(set_in, A);   // survivors: roots pass
                ent = en;
            } else if (PHASE != 1 && try_order(mt, L, A, e, nu, sg, tab, o)) {
                emit(sg, &cnt[s], k, o, st_loc, st_val);
            } else {
                if (step == 0 && ap > 0) wave_count(&cnt[s].mlp_fb, true);
                // general mode, rounds after the first: a hypothesis of order
                // 3 or 4 whose |c_0| pre-check failed (precheck_kernel, in
                // round 0) is skipped, as its round would reject it by the
                // same check on the same syndromes; one whose check passed
                // goes straight to the roots pass
                const unsigned pc = (!exact && round > 0) ? (unsigned)prechk[sg.bin_off + k] : 0u;
                int nx = step + 1, nord = 0;
                for (; nx < L; ++nx) {
                    nord = (ap > 0 && a0 == 0) ? 0 : seq_order(a0, ap, L, nx);
                    if (!((pc & 1u) && nord >= 3 && !(pc & (nord == 3 ? 2u : 4u)))) break;
                }
                if (nx < L) {
                    if (ap > 0 && a0 == 0) {
                        q = q_round(set_in ^ 1, 0);
                        ent = int2{s, pack_code(k, nx, ap, 0)};
                    } else {
                        q = ((pc & 1u) && nord >= 3) ? q_roots(set_in ^ 1, nord) : q_round(set_in ^ 1, nord);
                        ent = int2{s, pack_code(k, nx, ap, a0)};
                    }
                } else {
                    wave_count(&cnt[s].flagged, true);
                    if (!exact) {
                        q = q_cs(a0);
                        ent = int2{s, (int)k};
                    }
                }
            }
        }
        const int slot = bq.reserve(q);
        bq.commit(work, active, qlist, list_cap, q, slot, ent);
    }
}

// General mode, beside round 0: the |c_0| pre-checks (locator_check) of
// orders 3 and 4 for every bin queued for round 0, into prechk[bin] (bit 0:
// taken, bits 1 and 2: order 3 and 4 pass).  Bins whose round-0 order is 3
// or 4 get 0 (not taken): their pre-check is part of their rounds.
template <typename T>
__global__ __launch_bounds__(kBlock) void precheck_kernel(const SigDev* __restrict__ sigs,
                                                          const typename V2<T>::type* __restrict__ synd,
                                                          const WorkCounters* __restrict__ work,
                                                          const int2* __restrict__ qlist, int64_t list_cap,
                                                          unsigned char* __restrict__ prechk) {
    constexpr int kSeg = kMaxL;
    int start[kSeg + 1];
    start[0] = 0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) start[i + 1] = start[i] + work->q[q_round(0, i + 1)];
    const int total = start[kSeg];
    for (int item = blockIdx.x * kBlock + threadIdx.x; item < total; item += gridDim.x * kBlock) {
        int seg = 0;
#pragma unroll
        for (int i = 1; i < kSeg; ++i)
            if (item >= start[i]) seg = i;
        int s0 = start[0];
#pragma unroll
        for (int i = 1; i < kSeg; ++i)
            if (seg == i) s0 = start[i];
        const int2 en = qlist[(int64_t)q_round(0, seg + 1) * list_cap + (item - s0)];
        // by value: the fields are read together, not at their first use behind a branch
        const SigDev sg = sigs[en.x];
        if (sg.mode != kGeneral) continue;
        const int64_t k = code_k(en.y);
        unsigned pc = 0u;
        if (seg <= 1) {
            const int L = sg.L;
            zd mt[2 * kMaxL];
            load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
            derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
            zd cc[kMaxL];
            pc = 1u;
            if (L >= 3 && locator_check(mt, 3, sg, cc)) pc |= 2u;
            if (L >= 4 && locator_check(mt, 4, sg, cc)) pc |= 4u;
        }
        prechk[sg.bin_off + k] = (unsigned char)pc;
    }
}

// Plans without general-mode signals finish in one kernel what few bins
// remain after round 0 of orders 1 and 2: the bins of round 0 whose first
// order is 3 or 4 (set 0, slots 3..4), those of the later rounds (set 1,
// slots 1..4) and, in learned plans, the bins still without a rank order
// (set 1, slot 0: a failed predicted order, or no prediction), which take the
// rank test here first.  Each bin tries its remaining orders in turn (same
// sequence, same judge), is emitted at the first accepted one and flagged
// when none is left.
template <typename T>
__global__ __launch_bounds__(kBlock) void rest_kernel(const SigDev* __restrict__ sigs,
                                                      const typename V2<T>::type* __restrict__ synd,
                                                      const double2* __restrict__ tab, SigCounters* __restrict__ cnt,
                                                      int64_t* __restrict__ st_loc, double2* __restrict__ st_val,
                                                      const WorkCounters* __restrict__ work,
                                                      const int2* __restrict__ qlist, int64_t list_cap) {
    // the queues as one index space
    constexpr int kSeg = 3 + kMaxL;
    const int qs[kSeg] = {q_round(0, 3), q_round(0, 4), q_round(1, 0), q_round(1, 1),
                          q_round(1, 2), q_round(1, 3), q_round(1, 4)};
    int start[kSeg + 1];
    start[0] = 0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) start[i + 1] = start[i] + work->q[qs[i]];
    const int total = start[kSeg];
    for (int item = blockIdx.x * kBlock + threadIdx.x; item < total; item += gridDim.x * kBlock) {
        int seg = 0;
#pragma unroll
        for (int i = 1; i < kSeg; ++i)
            if (item >= start[i]) seg = i;
        int qid = qs[0];
#pragma unroll
        for (int i = 1; i < kSeg; ++i)
            if (seg == i) qid = qs[i];
        int s0 = start[0];
#pragma unroll
        for (int i = 1; i < kSeg; ++i)
            if (seg == i) s0 = start[i];
        const int2 en = qlist[(int64_t)qid * list_cap + (item - s0)];
        const int s = en.x;
        const int code = en.y;
        const int64_t k = code_k(code);
        const int ap = code_ap(code), a0 = code_a0(code);
        // by value: the fields are read together, not at their first use behind a branch
        const SigDev sg = sigs[s];
        const int L = sg.L;
        zd mt[2 * kMaxL];
        load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
        double e = 0.0;
#pragma unroll
        for (int l = 0; l < 2 * kMaxL; ++l) e += norm2(mt[l]);
        derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
        BinOut o;
        o.n = 0;
        bool done = false;
        int r0 = a0;
        for (int step = code_step(code); step < L && !done; ++step) {
            if (r0 == 0) {
                // no rank order yet (learned plans): the rank test
                if (rank_one_certified(mt, L, sg.tau_rank)) {
                    r0 = 1;
                } else {
                    double sv[kMaxL];
                    hankel_singular_values(mt, L, sv);
                    r0 = rank_order(sv, L, sg.tau_rank);
                }
            }
            // one constant-order copy per order: the same arithmetic as round_kernel<A>
            switch (seq_order(r0, ap, L, step)) {
                case 1: done = try_order(mt, L, 1, e, 0.0, sg, tab, o); break;
                case 2: done = try_order(mt, L, 2, e, 0.0, sg, tab, o); break;
                case 3: done = try_order(mt, L, 3, e, 0.0, sg, tab, o); break;
                default: done = try_order(mt, L, 4, e, 0.0, sg, tab, o); break;
            }
            if (!done && step == 0 && ap > 0) wave_count(&cnt[s].mlp_fb, true);
        }
        if (done) emit(sg, &cnt[s], k, o, st_loc, st_val);
        else wave_count(&cnt[s].flagged, true);
    }
}

__global__ void zero_set_kernel(WorkCounters* work, int set) {
    if (threadIdx.x < kRoundSlots) work->q[q_round(set, threadIdx.x)] = 0;
    if (threadIdx.x < 2) work->q[q_roots(set, 3 + threadIdx.x)] = 0;
}

// Lanes per bin of the CS step: order 1 needs no scan over the roots of
// unity; higher orders split it over a group of lanes, wider for the rarer
// orders, whose few bins would otherwise each be one lane's long serial chain.
__host__ __device__ constexpr int cs_group_lanes(int a0) { return a0 <= 1 ? 1 : a0 == 2 ? 1 : a0 == 3 ? 8 : 16; }

// CS step for the bins the decoder queued (general mode), one lane (or group
// of lanes) per bin; one instantiation per vote order A0, so every wave runs
// one code path.
template <typename T, int A0>
__global__ __launch_bounds__(kBlock) void cs_kernel(const SigDev* __restrict__ sigs,
                                                    const int64_t* __restrict__ shifts,
                                                    const typename V2<T>::type* __restrict__ synd,
                                                    const double2* __restrict__ tab,
                                                    const double2* __restrict__ gram, SigCounters* __restrict__ cnt,
                                                    int64_t* __restrict__ st_loc, double2* __restrict__ st_val,
                                                    const WorkCounters* __restrict__ work,
                                                    const int2* __restrict__ qlist, int64_t list_cap) {
    constexpr int G = cs_group_lanes(A0);
    const int gl = threadIdx.x & (G - 1);
    const int total = work->q[q_cs(A0)];
    const int2* in = qlist + (int64_t)q_cs(A0) * list_cap;
    for (int item = (blockIdx.x * kBlock + threadIdx.x) / G; item < total; item += gridDim.x * (kBlock / G)) {
        const int2 en = in[item];
        const int s = en.x;
        const int64_t k = en.y;
        // the signal's fields by value: read together here rather than one
        // at a time at their first use behind the branches below
        const SigDev sg = sigs[s];
        const int L = sg.L;
        const int64_t* sh = shifts + sg.shift_off;
        zd mt[2 * kMaxL];
        load_raw<T, 2 * kMaxL>(synd, sg, k, 2 * L, mt);
        derotate_consecutive<2 * kMaxL>(mt, k, sg.n, 2 * L);
        const int R = sg.R;
        const RowSource<T> ysrc{synd + synd_at(sg, 2 * L, k), sg.log2m, k, sg.n, sh + 2 * L};
        BinOut o;
        o.n = 0;
        const bool ok = cs_recover<A0, G>(mt, ysrc, R, sh + 2 * L, sg, tab, gram, o);
        if (!ok || gl != 0) o.n = 0;   // one lane of the group reports the bin
        wave_count(&cnt[s].cs, ok && gl == 0);
        emit(sg, &cnt[s], k, o, st_loc, st_val);
    }
}

// ------------------------------------------------------------ output lists

// Location sort of long lists (more than kRankChunk entries) by buckets of
// the location's high bits: counts per bucket, their exclusive scan (the
// bucket's first output position), the entries scattered into their
// buckets' ranges (any order within a range), then every entry's position =
// its range's start + the number of its range's locations below its own
// (locations within a signal are distinct).  About 4 entries per bucket for
// uniformly spread locations; a list with a bucket above kOutBucketMax
// entries is left to block_rank.
constexpr int kOutBuckets = 4096;
constexpr int kOutBucketMax = 256;
struct BucketLds {
    int base[kOutBuckets + 1];   // counts, then their exclusive scan
    int cur[kOutBuckets];        // scatter cursors
    int part[kRankThreads / 64];
    int maxc;
};

// Writes the sorted list (positions below cap) and returns true, or returns
// false (nothing written) when some bucket holds more than kOutBucketMax
// entries.  e_of(j) = staging index of list entry j < nk; tl / tj: scratch
// of nk locations / staging indices.  Whole block.
template <typename EntryFn>
__device__ bool bucket_sort_out(EntryFn e_of, int nk, const int64_t* __restrict__ loc, const double2* __restrict__ val,
                                int64_t n, BucketLds& B, long long* __restrict__ tl, int* __restrict__ tj, int64_t* o_loc,
                                double2* o_val, int64_t cap) {
    int lnb = 0;
    while ((1 << lnb) < kOutBuckets && (4 << lnb) < nk) ++lnb;   // about 4 entries per bucket
    const int log2n = __builtin_ctzll((unsigned long long)n);
    if (lnb > log2n) lnb = log2n;
    const int nb = 1 << lnb, shift = log2n - lnb;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) B.base[b] = 0;
    if (threadIdx.x == 0) B.maxc = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < nk; j += blockDim.x) atomicAdd(&B.base[(int)(loc[e_of(j)] >> shift)], 1);
    __syncthreads();
    // exclusive scan of the counts: each thread a contiguous run, wave then block partials
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
    int run = 0, mx = 0;
    for (int b = lo; b < hi; ++b) {
        run += B.base[b];
        mx = max(mx, B.base[b]);
    }
    if (mx > 0) atomicMax(&B.maxc, mx);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) B.part[wv] = inc;
    __syncthreads();
    int before = inc - run;
    for (int w = 0; w < wv; ++w) before += B.part[w];
    for (int b = lo; b < hi; ++b) {
        const int c = B.base[b];
        B.base[b] = before;
        B.cur[b] = before;
        before += c;
    }
    if (threadIdx.x == 0) B.base[nb] = nk;
    __syncthreads();
    if (B.maxc > kOutBucketMax) return false;   // uniform: read after the barrier
    for (int j = threadIdx.x; j < nk; j += blockDim.x) {
        const int e = e_of(j);
        const int64_t l = loc[e];
        const int pos = atomicAdd(&B.cur[(int)(l >> shift)], 1);
        tl[pos] = (long long)l;
        tj[pos] = e;
    }
    __syncthreads();   // the block's scratch writes are visible to the block
    for (int p = threadIdx.x; p < nk; p += blockDim.x) {
        const long long l = tl[p];
        const int b = (int)(l >> shift);
        const int q0 = B.base[b], q1 = B.base[b + 1];
        int r = q0;
        for (int q = q0; q < q1; ++q) r += tl[q] < l ? 1 : 0;
        if (r < cap) {
            o_loc[r] = (int64_t)l;
            o_val[r] = val[tj[p]];
        }
    }
    return true;
}

// One block per signal.  General mode keeps the K entries of largest |value|
// when more were found (ties to the lower location); iterative mode drops the
// entries marked cancelled; the kept entries are written sorted by location
// (locations within a signal are distinct).
__global__ __launch_bounds__(kRankThreads) void output_kernel(const SigDev* __restrict__ sigs, const IoDev* __restrict__ io,
                                                              SigCounters* __restrict__ cnt,
                                                              const int64_t* __restrict__ st_loc,
                                                              const double2* __restrict__ st_val, int* __restrict__ kidx,
                                                              double* rk_a, long long* rk_b, int* rk_i, int* rk_r) {
    // the location sort (LDS) and the radix selections of the top-K share one
    // region (40 KB: four blocks per CU)
    __shared__ union {
        RankLds rank;
        RadixLds radix;
        BucketLds bucket;
    } U;
    RankLds& S = U.rank;
    const int s = blockIdx.x;
    const SigDev& sg = sigs[s];
    const IoDev o = io[s];
    int n = cnt[s].stage_count;
    if (n > sg.stage_cap) n = sg.stage_cap;
    const int64_t* loc = st_loc + sg.stage_off;
    const double2* val = st_val + sg.stage_off;
    int* kx = kidx + sg.stage_off;
    const RankScratch g = rank_scratch(rk_a, rk_b, rk_i, rk_r, sg.stage_off);
    int& n_kept = U.radix.n_cand;   // keep counter of the paths that append
    int nk;
    if (sg.mode == kGeneral && n > sg.k_votes) {
        // the K first entries in order of (|value| desc, location asc): the
        // K-th largest |value|^2 by radix selection (key: complemented bits,
        // so ascending key = descending magnitude; NaN as zero), then, when
        // several entries share that magnitude, the lowest locations among
        // them by a second selection
        auto mag = [&](int i) -> unsigned long long {
            const double2 v = val[i];
            const double m = v.x * v.x + v.y * v.y;
            return ~(unsigned long long)__double_as_longlong(m == m ? m : 0.0);
        };
        const int ik = block_radix_select(mag, n, sg.k_votes - 1, U.radix);
        const unsigned long long uk = mag(ik);
        int& n_gt = U.radix.sel_digit;   // free between the selections
        int& n_eq = U.radix.sel_rr;
        if (threadIdx.x == 0) {
            n_gt = 0;
            n_eq = 0;
        }
        __syncthreads();
        int cg = 0, ce = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const unsigned long long ui = mag(i);
            cg += ui < uk ? 1 : 0;
            ce += ui == uk ? 1 : 0;
        }
        if (cg) atomicAdd(&n_gt, cg);
        if (ce) atomicAdd(&n_eq, ce);
        __syncthreads();
        const int need = sg.k_votes - n_gt;   // 1 <= need <= n_eq
        const int eq = n_eq;
        __syncthreads();                      // n_gt, n_eq read before the second selection reuses them
        int64_t lk = INT64_MAX;               // all entries of magnitude uk kept
        if (need < eq)
            lk = loc[block_radix_select([&](int i) { return mag(i) == uk ? (unsigned long long)loc[i] : ~0ull; }, n,
                                        need - 1, U.radix)];
        if (threadIdx.x == 0) n_kept = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const unsigned long long ui = mag(i);
            if (ui < uk || (ui == uk && loc[i] <= lk)) kx[atomicAdd(&n_kept, 1)] = i;
        }
        __syncthreads();
        nk = n_kept;
    } else if (sg.mode == kIterative) {
        // entries whose accumulated value cancelled carry location -1
        // (locations are distinct, so the order of kx does not matter)
        if (threadIdx.x == 0) n_kept = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if (loc[i] >= 0) kx[atomicAdd(&n_kept, 1)] = i;
        __syncthreads();
        nk = n_kept;
    } else {
        for (int i = threadIdx.x; i < n; i += blockDim.x) kx[i] = i;
        nk = n;
    }
    __syncthreads();   // kx complete; U is reused below
    if (nk <= kRankChunk) {
        // (location << 24 | entry) as one 64-bit key (location < 2^40, entry < 2^24):
        // the sorted position is the output position
        unsigned long long* K = reinterpret_cast<unsigned long long*>(S.a);
        const int P = pow2_at_least(nk);
#pragma unroll 4
        for (int j = threadIdx.x; j < P; j += blockDim.x)
            K[j] = j < nk ? ((unsigned long long)loc[kx[j]] << 24) | (unsigned long long)j : ~0ull;
        __syncthreads();
        lds_bitonic64(K, P);
        for (int r = threadIdx.x; r < nk && r < o.cap; r += blockDim.x) {
            const int e = kx[(int)(K[r] & 0xffffffull)];
            o.loc[r] = loc[e];
            o.val[r] = val[e];
        }
    } else if (!bucket_sort_out([&](int j) { return kx[j]; }, nk, loc, val, sg.n, U.bucket, g.b, g.idx, o.loc, o.val,
                                o.cap)) {
        __syncthreads();   // U is reused
        block_rank([&](int j) { return RankKey{0.0, (long long)loc[kx[j]]}; }, nk, S, g);
        for (int j = threadIdx.x; j < nk; j += blockDim.x) {
            const int r = g.rank[j];
            if (r < o.cap) {
                o.loc[r] = loc[kx[j]];
                o.val[r] = val[kx[j]];
            }
        }
    }
    if (threadIdx.x == 0) {
        *o.count = nk;
        cnt[s].kept = nk;
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
    hipLaunchKernelGGL(select_kernel, dim3(c.n_general), dim3(kRankThreads), 0, c.stream, c.sigs, c.general_sigs,
                       c.sigma, c.ebin, c.sel, c.rk_a, c.rk_b, c.rk_i, c.rk_r);
    return hipGetLastError();
}

hipError_t launch_output(const LaunchCtx& c) {
    if (c.n_sigs == 0) return hipSuccess;
    hipLaunchKernelGGL(output_kernel, dim3(c.n_sigs), dim3(kRankThreads), 0, c.stream, c.sigs, c.io, c.cnt, c.st_loc,
                       c.st_val, c.kidx, c.rk_a, c.rk_b, c.rk_i, c.rk_r);
    return hipGetLastError();
}

hipError_t launch_activity(const LaunchCtx& c) {
    if (c.n_act_items == 0) return hipSuccess;
    hipLaunchKernelGGL(activity_kernel, dim3(c.n_act_items), dim3(kBlock), 0, c.stream, c.sigs, c.act_items,
                       c.fp64 ? nullptr : (const float2*)c.synd, c.fp64 ? (const double2*)c.synd : nullptr, c.epart,
                       c.sigma, c.sel, c.work, c.active_list, c.qlist, c.list_cap, c.cnt);
    return hipGetLastError();
}

hipError_t launch_certify(const LaunchCtx& c) {
    if (c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(certify_kernel<double>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const double2*)c.synd, c.omega, c.cnt, c.st_loc, c.st_val, c.work, c.active_list, c.qlist,
                           c.list_cap);
    else
        hipLaunchKernelGGL(certify_kernel<float>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const float2*)c.synd, c.omega, c.cnt, c.st_loc, c.st_val, c.work, c.active_list, c.qlist,
                           c.list_cap);
    return hipGetLastError();
}

hipError_t launch_svd_rank(const LaunchCtx& c, int q_in, int set_out) {
    if (c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(svd_rank_kernel<double>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const double2*)c.synd, c.work, c.active_list, c.qlist, c.list_cap, q_in, set_out);
    else
        hipLaunchKernelGGL(svd_rank_kernel<float>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const float2*)c.synd, c.work, c.active_list, c.qlist, c.list_cap, q_in, set_out);
    return hipGetLastError();
}

hipError_t launch_zero_set(const LaunchCtx& c, int set) {
    hipLaunchKernelGGL(zero_set_kernel, dim3(1), dim3(64), 0, c.stream, c.work, set);
    return hipGetLastError();
}

template <typename T, int A, int PHASE>
static void launch_round_one(const LaunchCtx& c, int round) {
    using V = typename V2<T>::type;
    hipLaunchKernelGGL((round_kernel<T, A, PHASE>), dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs, c.shifts,
                       (const V*)c.synd, c.sel, c.omega, c.cnt, c.st_loc, c.st_val, c.work, c.active_list, c.qlist,
                       c.list_cap, round, c.prechk);
}

// Orders 3 and 4 in two passes when the plan has general-mode signals (most
// of their hypotheses fail the |c_0| check); one fused pass otherwise.
template <typename T, int A>
static void launch_order(const LaunchCtx& c, int round) {
    if constexpr (A >= 3) {
        if (c.any_general) {
            launch_round_one<T, A, 1>(c, round);
            launch_round_one<T, A, 2>(c, round);
            return;
        }
    }
    launch_round_one<T, A, 0>(c, round);
}

template <typename T>
static void launch_round_t(const LaunchCtx& c, int round, int a) {
    // plans without general-mode signals leave round 0 of orders 3 and 4 to rest_kernel
    if (round == 0 && !c.any_general && a >= 3) return;
    if (a > c.max_l) return;
    switch (a) {
        case 1: launch_order<T, 1>(c, round); break;
        case 2: launch_order<T, 2>(c, round); break;
        case 3: launch_order<T, 3>(c, round); break;
        default: launch_order<T, 4>(c, round); break;
    }
}

hipError_t launch_precheck(const LaunchCtx& c) {
    if (!c.any_general || c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(precheck_kernel<double>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const double2*)c.synd, c.work, c.qlist, c.list_cap, c.prechk);
    else
        hipLaunchKernelGGL(precheck_kernel<float>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const float2*)c.synd, c.work, c.qlist, c.list_cap, c.prechk);
    return hipGetLastError();
}

hipError_t launch_rest(const LaunchCtx& c) {
    if (c.n_bin_items == 0) return hipSuccess;
    if (c.fp64)
        hipLaunchKernelGGL(rest_kernel<double>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const double2*)c.synd, c.omega, c.cnt, c.st_loc, c.st_val, c.work, c.qlist, c.list_cap);
    else
        hipLaunchKernelGGL(rest_kernel<float>, dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const float2*)c.synd, c.omega, c.cnt, c.st_loc, c.st_val, c.work, c.qlist, c.list_cap);
    return hipGetLastError();
}

hipError_t launch_round(const LaunchCtx& c, int round, int a) {
    if (c.n_bin_items == 0) return hipSuccess;
    if (c.fp64) launch_round_t<double>(c, round, a);
    else launch_round_t<float>(c, round, a);
    return hipGetLastError();
}

template <typename T, int A0>
static void launch_cs_one(const LaunchCtx& c) {
    using V = typename V2<T>::type;
    hipLaunchKernelGGL((cs_kernel<T, A0>), dim3(c.n_work_blocks), dim3(kBlock), 0, c.stream, c.sigs, c.shifts,
                       (const V*)c.synd, c.omega, c.gram, c.cnt, c.st_loc, c.st_val, c.work, c.qlist, c.list_cap);
}

hipError_t launch_cs(const LaunchCtx& c, int a0) {
    if (!c.any_general || c.n_bin_items == 0) return hipSuccess;
    if (c.fp64) {
        switch (a0) {
            case 1: launch_cs_one<double, 1>(c); break;
            case 2: launch_cs_one<double, 2>(c); break;
            case 3: launch_cs_one<double, 3>(c); break;
            default: launch_cs_one<double, 4>(c); break;
        }
    } else {
        switch (a0) {
            case 1: launch_cs_one<float, 1>(c); break;
            case 2: launch_cs_one<float, 2>(c); break;
            case 3: launch_cs_one<float, 3>(c); break;
            default: launch_cs_one<float, 4>(c); break;
        }
    }
    return hipGetLastError();
}

}  // namespace sft
