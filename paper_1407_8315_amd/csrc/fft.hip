// Step 1-2 of sFFT-DT on the device: strided downsampling at each shift and
// the length-M FFT of every downsampled signal, scaled by d:
//     m_l[k] = d * sum_{k'} x[(d k' + l) mod N] e^{-2 pi i k k' / M}
// (Sec. II-A, x_{d,l}[k] = x[dk + l]; Alg. 1 "FFT(x_{d,l}) x d"; Alg. 2 Part 1).
//
// One block handles `nlines` shifts of one signal (nlines * M <= points held in
// LDS).  The gather reads the shifts of a block with the shift index fastest,
// so consecutive shifts (the 2L consecutive l of a bin group) form contiguous
// runs of 8 * nlines bytes.  Blocks of one signal are ordered so that they land
// on the same XCD (block ids of a signal share their residue mod 8 and are
// adjacent in dispatch order), letting that XCD's L2 serve the other shifts'
// bytes of each fetched line.
//
// FFT: Stockham auto-sort passes of radix 16 (then one pass of 8, 4 or 2 for
// the remaining factor) over every line held in LDS.  Each thread loads the
// inputs of its butterflies into registers, the block synchronises, and the
// thread writes the outputs back, so a single LDS buffer suffices.
#include "common.h"

namespace sft {

constexpr int kGatherBatch = 16;   // strided loads in flight per thread

template <typename T>
struct C2;
template <>
struct C2<float> {
    using type = float2;
};
template <>
struct C2<double> {
    using type = double2;
};

template <typename V>
__device__ inline V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V>
__device__ inline V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V>
__device__ inline V cmulv(V a, V b) { return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename V>
__device__ inline V mul_mi(V a) { return V{a.y, -a.x}; }   // a * (-i)

// In-register forward DFT of R points (R = 2, 4, 8, 16), by radix-2 splits.
template <typename V, int R>
struct Dft;
template <typename V>
struct Dft<V, 2> {
    __device__ static inline void run(V* v) {
        V a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <typename V>
struct Dft<V, 4> {
    __device__ static inline void run(V* v) {
        V s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        V s13 = cadd(v[1], v[3]), d13 = mul_mi(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    }
};
template <typename V, int R>
struct Dft {
    __device__ static inline void run(V* v) {
        constexpr int H = R / 2;
        V e[H], o[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<V, H>::run(e);
        Dft<V, H>::run(o);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            // w_R^{-k} = cos(2 pi k / R) - i sin(2 pi k / R)
            using S = decltype(v[0].x);
            const S c = (S)__builtin_cos(2.0 * M_PI * k / R);
            const S s = (S)__builtin_sin(2.0 * M_PI * k / R);
            V t = cmulv(o[k], V{c, -s});
            v[k] = cadd(e[k], t);
            v[k + H] = csub(e[k], t);
        }
    }
};

// One Stockham pass of radix R over `nlines` lines of length M (= 2^log2m)
// held line-major in buf; Ns = product of the radices of earlier passes.
template <typename T, int R, int PMAX>
__device__ inline void stockham_pass(typename C2<T>::type* buf, int log2m, int nlines, int log2ns,
                                     const typename C2<T>::type* tw, int tw_log2) {
    using V = typename C2<T>::type;
    constexpr int LOG2R = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
    constexpr int Q = (PMAX / R + kBlock - 1) / kBlock;
    const int log2mr = log2m - LOG2R;
    const int B = nlines << log2mr;
    const int ns = 1 << log2ns;
    V v[Q][R];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int b = threadIdx.x + q * kBlock;
        if (b < B) {
            int line = b >> log2mr, j = b & ((1 << log2mr) - 1);
            const V* src = buf + ((size_t)line << log2m) + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = src[r << log2mr];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        int b = threadIdx.x + q * kBlock;
        if (b < B) {
            int line = b >> log2mr, j = b & ((1 << log2mr) - 1);
            int k = j & (ns - 1);
            if (ns > 1) {
                // twiddle w_{ns R}^{-r k} = tw[r k 2^tw_log2 / (ns R)]
                const int sh = tw_log2 - (log2ns + LOG2R);
#pragma unroll
                for (int r = 1; r < R; ++r) v[q][r] = cmulv(v[q][r], tw[(r * k) << sh]);
            }
            Dft<V, R>::run(v[q]);
            V* dst = buf + ((size_t)line << log2m) + (((j >> log2ns) << (log2ns + LOG2R)) + k);
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r << log2ns] = v[q][r];
        }
    }
    __syncthreads();
}

// One block = `nl` lines of one signal held in LDS, transformed in place.
// pass 0 (M fits one block): line = shift s, gathered from x at stride d,
//   output m_s[k] = d * X[k] -> syndromes [s][k], plus the line energy.
// pass 1 (first of two, M = M1 * M2): line = (s, n1), the M2 samples
//   x[(d (n1 + M1 n2) + shift_s) mod N]; output Y[s][k2][n1] = X[k2] w_M^{-n1 k2}.
// pass 2: line = (s, k2), the M1 values Y[s][k2][.]; output
//   m_s[k2 + M2 k1] = d * X[k1] -> syndromes.
template <typename T, int PMAX, typename TIN>
__global__ __launch_bounds__(kBlock) void syndrome_kernel(const SigDev* __restrict__ sigs, const IoDev* __restrict__ io,
                                                          const int4* __restrict__ items, const int64_t* __restrict__ shifts,
                                                          const typename C2<T>::type* __restrict__ tw, int tw_log2,
                                                          typename C2<T>::type* __restrict__ synd,
                                                          typename C2<T>::type* __restrict__ ybuf,
                                                          double* __restrict__ epart, SigCounters* __restrict__ cnt) {
    using V = typename C2<T>::type;
    __shared__ V buf[PMAX];
    __shared__ double red[kBlock];
    const int4 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const int s = it.x, line0 = it.y, nl = it.z, pass = it.w;
    const SigDev sg = sigs[s];
    using VIN = typename C2<TIN>::type;   // input element (complex64 or complex128)
    const VIN* __restrict__ x = reinterpret_cast<const VIN*>(io[sg.parent].x);
    const int log2m = sg.log2m;
    const int log2m1 = sg.log2m1, log2m2 = log2m - log2m1;
    const int log2len = pass == 0 ? log2m : (pass == 1 ? log2m2 : log2m1);
    const int len = 1 << log2len;
    const int64_t nmask = sg.n - 1;
    const int64_t* sh = shifts + sg.shift_off;

    // gather into LDS, line-major [line][j]
    int bad = 0;
    const int P = nl << log2len;
    if (pass == 2) {
        // contiguous rows of the intermediate: position fastest
        const V* y = ybuf + sg.y_off;
        for (int p = threadIdx.x; p < P; p += kBlock) {
            const int line = p >> log2len, j = p & (len - 1);
            buf[p] = y[((int64_t)(line0 + line) << log2m1) + j];
        }
    } else {
        // strided samples of x: line fastest, so consecutive shifts read adjacent
        // samples.  kGatherBatch loads per thread are issued before any is
        // stored, so that many requests are in flight per wave.
        // p / nl by multiply-high: exact for p < 2^32 / nl (here p < 2^14, nl <= 2^7).
        const unsigned long long inv = (0xFFFFFFFFull + (unsigned)nl) / (unsigned)nl;
        for (int p0 = threadIdx.x; p0 < P; p0 += kGatherBatch * kBlock) {
            V v[kGatherBatch];
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                const int p = p0 + u * kBlock;
                if (p < P) {
                    const int j = (int)(((unsigned long long)p * inv) >> 32);
                    const int g = line0 + (p - j * nl);
                    int64_t idx;
                    if (pass == 0) {
                        idx = (sg.d * (int64_t)j + sh[g]) & nmask;
                    } else {
                        const int l = g >> log2m1, n1 = g & ((1 << log2m1) - 1);
                        idx = (sg.d * ((int64_t)n1 + ((int64_t)j << log2m1)) + sh[l]) & nmask;
                    }
                    const VIN xi = x[idx];
                    v[u].x = (T)xi.x;
                    v[u].y = (T)xi.y;
                }
            }
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                const int p = p0 + u * kBlock;
                if (p < P) {
                    const int j = (int)(((unsigned long long)p * inv) >> 32);
                    const int line = p - j * nl;
                    if (sg.flags & 4) bad += !(isfinite(v[u].x) && isfinite(v[u].y));
                    buf[(line << log2len) + j] = v[u];
                }
            }
        }
        if ((sg.flags & 4) && bad) atomicAdd(&cnt[sg.parent].nonfinite, bad);
    }
    __syncthreads();

    // Stockham passes: radix 16 while >= 4 bits remain, then 8, 4 or 2
    int log2ns = 0;
    while (log2len - log2ns >= 4) {
        stockham_pass<T, 16, PMAX>(buf, log2len, nl, log2ns, tw, tw_log2);
        log2ns += 4;
    }
    switch (log2len - log2ns) {
        case 3: stockham_pass<T, 8, PMAX>(buf, log2len, nl, log2ns, tw, tw_log2); break;
        case 2: stockham_pass<T, 4, PMAX>(buf, log2len, nl, log2ns, tw, tw_log2); break;
        case 1: stockham_pass<T, 2, PMAX>(buf, log2len, nl, log2ns, tw, tw_log2); break;
        default: break;
    }

    const T dscale = (T)sg.d;
    if (pass == 0) {
        // scale by d, store, per-line energy (FP64, fixed-order tree)
        for (int line = 0; line < nl; ++line) {
            double acc = 0.0;
            for (int k = threadIdx.x; k < len; k += kBlock) {
                V v = buf[(line << log2m) + k];
                v.x *= dscale;
                v.y *= dscale;
                synd[synd_at(sg, line0 + line, k)] = v;
                acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            }
            red[threadIdx.x] = acc;
            __syncthreads();
            for (int w = kBlock / 2; w > 0; w >>= 1) {
                if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) epart[sg.epart_off + line0 + line] = red[0];
            __syncthreads();
        }
    } else if (pass == 1) {
        // twiddle w_M^{-n1 k2}, store Y[l][k2][n1] (lines = consecutive n1: contiguous)
        V* y = ybuf + sg.y_off;
        const int mtw = tw_log2 - log2m;
        for (int q = threadIdx.x; q < P; q += kBlock) {
            const int line = q % nl, k2 = q / nl;
            const int g = line0 + line;
            const int l = g >> log2m1, n1 = g & ((1 << log2m1) - 1);
            V v = buf[(line << log2len) + k2];
            const int64_t e = ((int64_t)n1 * k2) & ((1ll << log2m) - 1);
            v = cmulv(v, tw[e << mtw]);
            y[((((int64_t)l << log2m2) + k2) << log2m1) + n1] = v;
        }
    } else {
        // m_l[k2 + M2 k1] = d X[k1] (lines = consecutive k2: contiguous)
        for (int q = threadIdx.x; q < P; q += kBlock) {
            const int line = q % nl, k1 = q / nl;
            const int g = line0 + line;
            const int l = g >> log2m2, k2 = g & ((1 << log2m2) - 1);
            V v = buf[(line << log2len) + k1];
            v.x *= dscale;
            v.y *= dscale;
            synd[synd_at(sg, l, k2 + ((int64_t)k1 << log2m2))] = v;
        }
    }
}

// Consecutive-shift lines of FP32 units with 2^8 <= M <= 2^12 points (the
// 2L consecutive shifts of exact- and general-mode signals, the two shifts of
// an iterative grid): one block holds P line pairs (lines line0 .. line0+2P-1,
// shifts sh[line0] + 0 .. 2P-1) of one unit, with T = M / PT threads per pair
// (PT = 2^LPT points of each line per thread).  Thread (p, j), p < P, j < T,
// with p fastest so that the P lanes reading one 64 B run of 2P consecutive
// samples sit next to each other in the wave, loads the samples
// d (j + T s) + shift, s < PT, of its two lines as one 16-byte load each: a
// block touches every fetched run once (the one-line-per-block kernel above
// requests it once per line).
//
// FFT (the Stockham passes of stockham_pass, radix PT, then one of a smaller
// power of two): in every pass, thread j takes the PT points j + T s of a line
// (one butterfly of radix PT, or PT/R of radix R); the first pass runs on the
// gathered registers, every later pass reads its inputs from LDS, where the
// previous pass wrote its outputs; the last pass leaves X[j + T s] in
// registers.  The LDS holds one line of each pair at a time (both lines of a
// pair share the butterflies and twiddles), padded by one point per 16
// against bank conflicts, plus the twiddles w_M^e for e <= M/8 (the others
// follow exactly by symmetry).
template <int LOG2M, int LPT>
struct PairFft {
    static constexpr int M = 1 << LOG2M;
    static constexpr int PT = 1 << LPT;
    static constexpr int T = M / PT;
    static constexpr int NPASS = (LOG2M + LPT - 1) / LPT;
    static constexpr int lds_points() { return M + M / 16; }
    __device__ static inline int pad(int i) { return i + (i >> 4); }
    __host__ __device__ static constexpr int log2r(int pass) { return pass < LOG2M / LPT ? LPT : LOG2M - LPT * pass; }
};

// w_M^e, 0 <= e < M, from the table q[e'] = w_M^{e'}, e' <= M/8: within a
// quarter, w_M^{M/4 - e'} = -i conj(w_M^{e'}); across quarters, powers of -i
// (every step exact).
template <int LOG2M>
__device__ inline float2 twiddle_q(const float2* q, int e) {
    constexpr int Q = 1 << (LOG2M - 2);
    const int e0 = e & (Q - 1);
    float2 w;
    if (e0 <= Q / 2) {
        w = q[e0];
    } else {
        const float2 t = q[Q - e0];
        w = float2{-t.y, -t.x};
    }
    switch (e >> (LOG2M - 2)) {
        case 0: return w;
        case 1: return float2{w.y, -w.x};    // * (-i)
        case 2: return float2{-w.x, -w.y};   // * (-1)
        default: return float2{-w.y, w.x};   // * (+i)
    }
}

// One Stockham pass of radix 2^LR with ns = 2^LNS on the PT points a thread
// holds (v[s] = point j + T s); writes its outputs to `lds` (padded line)
// unless it is the last pass, which leaves X[j + T s] in v[s].
template <int LOG2M, int LPT, int LR, int LNS, bool LAST>
__device__ inline void pair_pass(float2 (&v)[1 << LPT], int j, const float2* qtw, float2* lds, bool on) {
    using F = PairFft<LOG2M, LPT>;
    constexpr int R = 1 << LR, NB = F::PT / R;
    if (!on) return;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = j + F::T * q;           // butterfly index
        const int k = b & ((1 << LNS) - 1);
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q + NB * r];
        if (LNS > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = cmulv(u[r], twiddle_q<LOG2M>(qtw, (r * k) << (LOG2M - LNS - LR)));
        }
        Dft<float2, R>::run(u);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q + NB * r] = u[r];
        } else {
            const int base = ((b >> LNS) << (LNS + LR)) + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[F::pad(base + (r << LNS))] = u[r];
        }
    }
}

// Passes 1 .. NPASS-1 of one line through LDS (pass 0 already written there).
// Threads with on = false (beyond the line's T) only take part in the
// barriers.
template <int LOG2M, int LPT, int PASS>
__device__ inline void pair_rest(float2 (&v)[1 << LPT], int j, const float2* qtw, float2* lds, bool on) {
    using F = PairFft<LOG2M, LPT>;
    if constexpr (PASS < F::NPASS) {
        __syncthreads();
        if (on) {
#pragma unroll
            for (int s = 0; s < F::PT; ++s) v[s] = lds[F::pad(j + F::T * s)];
        }
        __syncthreads();
        constexpr int LR = F::log2r(PASS);
        constexpr int LNS = LPT * PASS;   // every earlier pass was of radix PT
        pair_pass<LOG2M, LPT, LR, LNS, PASS == F::NPASS - 1>(v, j, qtw, lds, on);
        pair_rest<LOG2M, LPT, PASS + 1>(v, j, qtw, lds, on);
    }
}

// One line: pass 0 (radix PT, no twiddles) on the registers, the rest through
// LDS; leaves X[j + T s] in v[s].
template <int LOG2M, int LPT>
__device__ inline void pair_fft(float2 (&v)[1 << LPT], int j, const float2* qtw, float2* lds, bool on = true) {
    pair_pass<LOG2M, LPT, LPT, 0, false>(v, j, qtw, lds, on);
    pair_rest<LOG2M, LPT, 1>(v, j, qtw, lds, on);
}

// Scale by d in place and return the line's energy summed over the
// P-strided lanes of the wave (fixed order).
template <int P, int LPT>
__device__ inline double pair_scale_energy(float2 (&v)[1 << LPT], float dscale) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < (1 << LPT); ++s) {
        v[s].x *= dscale;
        v[s].y *= dscale;
        acc += (double)v[s].x * (double)v[s].x + (double)v[s].y * (double)v[s].y;
    }
    // lanes of the same p differ in the lane bits above log2 P
#pragma unroll
    for (int o = 32; o >= P; o >>= 1) acc += __shfl_xor(acc, o);
    return acc;
}

template <int P, int LOG2M, int LPT>
__global__ __launch_bounds__(P * (1 << (LOG2M - LPT))) void pair_syndrome_kernel(
    const SigDev* __restrict__ sigs, const IoDev* __restrict__ io, const int4* __restrict__ items,
    const int64_t* __restrict__ shifts, const float2* __restrict__ tw, int tw_log2, float2* __restrict__ synd,
    double* __restrict__ epart, SigCounters* __restrict__ cnt) {
    using F = PairFft<LOG2M, LPT>;
    constexpr int NT = P * F::T;
    static_assert(NT >= 64 && NT <= 1024, "whole waves, at most 1024 threads");
    __shared__ float2 lds[P][F::lds_points()];
    __shared__ float2 qtw[F::M / 8 + 1];
    __shared__ double red[NT / 64][2 * P];
    const int4 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const SigDev sg = sigs[it.x];
    const int line0 = it.y;
    const int p = threadIdx.x % P, j = threadIdx.x / P;
    const int64_t shift = shifts[sg.shift_off + line0] + 2 * p;   // shifts of lines line0 + 2p, +1
    const float2* __restrict__ x = reinterpret_cast<const float2*>(io[sg.parent].x);

    // gather: PT samples of each of the thread's two lines; d k' + shift + 1 < N (no wrap)
    float2 a[F::PT], b[F::PT];
    if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const float4* __restrict__ x4 = reinterpret_cast<const float4*>(x) + ((sg.d * (int64_t)j + shift) >> 1);
        const int64_t step = (sg.d * F::T) >> 1;   // T samples of stride d, in 16-byte units
#pragma unroll
        for (int s = 0; s < F::PT; ++s) {
            const float4 w = x4[s * step];
            a[s] = float2{w.x, w.y};
            b[s] = float2{w.z, w.w};
        }
    } else {
#pragma unroll
        for (int s = 0; s < F::PT; ++s) {
            const int64_t idx = sg.d * (int64_t)(j + F::T * s) + shift;
            a[s] = x[idx];
            b[s] = x[idx + 1];
        }
    }
    if (sg.flags & 4) {
        int bad = 0;
#pragma unroll
        for (int s = 0; s < F::PT; ++s)
            bad += !(isfinite(a[s].x) && isfinite(a[s].y)) + !(isfinite(b[s].x) && isfinite(b[s].y));
        if (bad) atomicAdd(&cnt[sg.parent].nonfinite, bad);
    }
    for (int e = threadIdx.x; e <= F::M / 8; e += NT) qtw[e] = tw[(int64_t)e << (tw_log2 - LOG2M)];

    const float dscale = (float)sg.d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    pair_fft<LOG2M, LPT>(a, j, qtw, lds[p], true);
    double acc = pair_scale_energy<P, LPT>(a, dscale);
    if (lane < P) red[wave][2 * lane] = acc;
    pair_fft<LOG2M, LPT>(b, j, qtw, lds[p], true);
    acc = pair_scale_energy<P, LPT>(b, dscale);
    if (lane < P) red[wave][2 * lane + 1] = acc;
    const int line = line0 + 2 * p;
    if (sg.bstride) {
        // by bin: the pair's two values of bin k side by side, one 16-byte store
        // (bstride and line even)
        float4* __restrict__ out = reinterpret_cast<float4*>(synd + synd_at(sg, line, 0));
#pragma unroll
        for (int s = 0; s < F::PT; ++s)
            out[((int64_t)(j + F::T * s) * sg.bstride) >> 1] = float4{a[s].x, a[s].y, b[s].x, b[s].y};
    } else {
        float2* __restrict__ out = synd + synd_at(sg, line, 0);
#pragma unroll
        for (int s = 0; s < F::PT; ++s) {
            out[j + F::T * s] = a[s];
            out[F::M + j + F::T * s] = b[s];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * P) {
        double e = 0.0;
        for (int w = 0; w < NT / 64; ++w) e += red[w][threadIdx.x];
        epart[sg.epart_off + line0 + 2 * (threadIdx.x >> 1) + (threadIdx.x & 1)] = e;
    }
}

// Iterative signals: the two lines of one grid M_l = M_0 / 2^l per block, in
// one launch for every grid of the signals of one M_0 (LOG2M0 = log2 M_0;
// grid l uses the first M_l / 8 threads of the block, the others take part in
// the barriers only).  Grid l reads x[d_l k' + 2l] and x[d_l k' + 2l + 1],
// d_l = 2^l d_0: the 16 bytes 16 l past x[d_0 (2^l k')], in a 128-byte line
// that grid 0 reads too; the blocks of a signal's grids are dispatched
// together on one XCD, so that its L2 serves the line to all of them.
template <int LOG2M, int LOG2M0>
__device__ inline void iter_grid(const SigDev& sg, const float2* __restrict__ x, int64_t shift, const float2* __restrict__ tw,
                                 int tw_log2, float2* __restrict__ synd, double* __restrict__ epart, SigCounters* cnt,
                                 float2* lds, float2* qtw, double (*red)[2]) {
    using F = PairFft<LOG2M, kPairLpt>;
    constexpr int NT = 1 << (LOG2M0 - kPairLpt);
    const int j = threadIdx.x;
    const bool on = j < F::T;
    float2 a[F::PT], b[F::PT];
#pragma unroll
    for (int s = 0; s < F::PT; ++s) a[s] = b[s] = float2{0.0f, 0.0f};
    if (on) {
        if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {   // shift even: 16-byte pairs
            const float4* __restrict__ x4 = reinterpret_cast<const float4*>(x) + ((sg.d * (int64_t)j + shift) >> 1);
            const int64_t step = (sg.d * F::T) >> 1;
#pragma unroll
            for (int s = 0; s < F::PT; ++s) {
                const float4 w = x4[s * step];
                a[s] = float2{w.x, w.y};
                b[s] = float2{w.z, w.w};
            }
        } else {
#pragma unroll
            for (int s = 0; s < F::PT; ++s) {
                const int64_t idx = sg.d * (int64_t)(j + F::T * s) + shift;
                a[s] = x[idx];
                b[s] = x[idx + 1];
            }
        }
        if (sg.flags & 4) {
            int bad = 0;
#pragma unroll
            for (int s = 0; s < F::PT; ++s)
                bad += !(isfinite(a[s].x) && isfinite(a[s].y)) + !(isfinite(b[s].x) && isfinite(b[s].y));
            if (bad) atomicAdd(&cnt[sg.parent].nonfinite, bad);
        }
    }
    __syncthreads();   // the previous grid is done with lds, qtw and red
    for (int e = j; e <= F::M / 8; e += NT) qtw[e] = tw[(int64_t)e << (tw_log2 - LOG2M)];
    const float dscale = (float)sg.d;
    const int lane = j & 63, wave = j >> 6;
    pair_fft<LOG2M, kPairLpt>(a, j, qtw, lds, on);
    double acc = pair_scale_energy<1, kPairLpt>(a, dscale);
    if (lane == 0) red[wave][0] = acc;
    pair_fft<LOG2M, kPairLpt>(b, j, qtw, lds, on);
    acc = pair_scale_energy<1, kPairLpt>(b, dscale);
    if (lane == 0) red[wave][1] = acc;
    if (on) {
        float2* __restrict__ out = synd + synd_at(sg, 0, 0);
#pragma unroll
        for (int s = 0; s < F::PT; ++s) {
            out[j + F::T * s] = a[s];
            out[F::M + j + F::T * s] = b[s];
        }
    }
    __syncthreads();
    if (j < 2) {
        double e = 0.0;
        for (int w = 0; w < (NT + 63) / 64; ++w) e += red[w][j];
        epart[sg.epart_off + j] = e;
    }
}

template <int LOG2M0>
__global__ __launch_bounds__(1 << (LOG2M0 - kPairLpt)) void iter_pair_kernel(
    const SigDev* __restrict__ sigs, const IoDev* __restrict__ io, const int4* __restrict__ items,
    const int64_t* __restrict__ shifts, const float2* __restrict__ tw, int tw_log2, float2* __restrict__ synd,
    double* __restrict__ epart, SigCounters* __restrict__ cnt) {
    constexpr int NT = 1 << (LOG2M0 - kPairLpt);
    static_assert(NT >= 64 && NT <= 1024, "whole waves, at most 1024 threads");
    __shared__ float2 lds[PairFft<LOG2M0, kPairLpt>::lds_points()];
    __shared__ float2 qtw[(1 << LOG2M0) / 8 + 1];
    __shared__ double red[NT / 64][2];
    const int4 it = items[blockIdx.x];
    if (it.x < 0) return;   // padding item
    const SigDev sg = sigs[it.x];   // the grid's view
    const float2* __restrict__ x = reinterpret_cast<const float2*>(io[sg.parent].x);
    const auto grid = [&](auto lg) {
        constexpr int LG = decltype(lg)::value;
        if constexpr (LG >= kPairLog2MMin)
            iter_grid<LG, LOG2M0>(sg, x, shifts[sg.shift_off], tw, tw_log2, synd, epart, cnt, lds, qtw, red);
    };
    switch (it.y) {   // l, uniform over the block
        case 0: grid(std::integral_constant<int, LOG2M0>{}); break;
        case 1: grid(std::integral_constant<int, LOG2M0 - 1>{}); break;
        case 2: grid(std::integral_constant<int, LOG2M0 - 2>{}); break;
        default: grid(std::integral_constant<int, LOG2M0 - 3>{}); break;
    }
}

// Line energies of two-pass signals: one block per (signal, line), fixed-order
// FP64 reduction (the one-pass kernel computes them in its epilogue).
template <typename T>
__global__ __launch_bounds__(kBlock) void line_energy_kernel(const SigDev* __restrict__ sigs, const int2* __restrict__ items,
                                                             const typename C2<T>::type* __restrict__ synd,
                                                             double* __restrict__ epart) {
    __shared__ double red[kBlock];
    const int2 it = items[blockIdx.x];
    const SigDev& sg = sigs[it.x];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < sg.m; k += kBlock) {
        auto v = synd[synd_at(sg, it.y, k)];
        acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[sg.epart_off + it.y] = red[0];
}

// sft_syndromes: the S lines of unit 0 as [S][M], whatever the layout.
template <typename V>
__global__ void copy_syndromes_kernel(const SigDev* __restrict__ sigs, const V* __restrict__ synd, V* __restrict__ out) {
    const SigDev& sg = sigs[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)sg.S << sg.log2m) return;
    const int line = (int)(i >> sg.log2m);
    const int64_t k = i & (sg.m - 1);
    out[i] = synd[synd_at(sg, line, k)];
}

hipError_t launch_copy_syndromes(const LaunchCtx& c, int64_t elems, void* out) {
    const int blocks = (int)((elems + kBlock - 1) / kBlock);
    if (c.fp64)
        hipLaunchKernelGGL(copy_syndromes_kernel<double2>, dim3(blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const double2*)c.synd, (double2*)out);
    else
        hipLaunchKernelGGL(copy_syndromes_kernel<float2>, dim3(blocks), dim3(kBlock), 0, c.stream, c.sigs,
                           (const float2*)c.synd, (float2*)out);
    return hipGetLastError();
}

__global__ void zero_counters_kernel(SigCounters* cnt, int n, WorkCounters* work) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = SigCounters{};
    if (i < (int)(sizeof(WorkCounters) / sizeof(int))) reinterpret_cast<int*>(work)[i] = 0;
}

hipError_t launch_zero_counters(const LaunchCtx& c) {
    int blocks = (c.n_sigs + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(blocks), dim3(kBlock), 0, c.stream, c.cnt, c.n_sigs, c.work);
    return hipGetLastError();
}

template <int P, int LOG2M>
static void launch_pair_group(const LaunchCtx& c) {
    const int g = pair_group(P, LOG2M);
    if (c.pair_n[g] == 0) return;
    constexpr int NT = P * (1 << (LOG2M - kPairLpt));
    if constexpr (NT >= 64 && NT <= 1024)
        hipLaunchKernelGGL((pair_syndrome_kernel<P, LOG2M, kPairLpt>), dim3(c.pair_n[g]), dim3(NT), 0, c.stream, c.sigs,
                           c.io, c.pair_items + c.pair_off[g], c.shifts, (const float2*)c.twiddle, c.tw_log2,
                           (float2*)c.synd, c.epart, c.cnt);
}

template <int P>
static void launch_pair_sizes(const LaunchCtx& c) {
    launch_pair_group<P, 8>(c);
    launch_pair_group<P, 9>(c);
    launch_pair_group<P, 10>(c);
    launch_pair_group<P, 11>(c);
    launch_pair_group<P, 12>(c);
}

template <int LOG2M0>
static void launch_iter_group(const LaunchCtx& c) {
    const int g = pair_group(0, LOG2M0);
    if (c.pair_n[g] == 0) return;
    constexpr int NT = 1 << (LOG2M0 - kPairLpt);
    if constexpr (NT >= 64 && NT <= 1024)
        hipLaunchKernelGGL((iter_pair_kernel<LOG2M0>), dim3(c.pair_n[g]), dim3(NT), 0, c.stream, c.sigs, c.io,
                           c.pair_items + c.pair_off[g], c.shifts, (const float2*)c.twiddle, c.tw_log2,
                           (float2*)c.synd, c.epart, c.cnt);
}

static void launch_pairs(const LaunchCtx& c) {
    launch_pair_sizes<1>(c);
    launch_pair_sizes<2>(c);
    launch_pair_sizes<4>(c);
    launch_iter_group<9>(c);
    launch_iter_group<10>(c);
    launch_iter_group<11>(c);
    launch_iter_group<12>(c);
}

template <int PMAX>
static void launch_f32_items(const LaunchCtx& c, const int4* items, int n) {
    if (n)
        hipLaunchKernelGGL((syndrome_kernel<float, PMAX, float>), dim3(n), dim3(kBlock), 0, c.stream, c.sigs, c.io, items,
                           c.shifts, (const float2*)c.twiddle, c.tw_log2, (float2*)c.synd, (float2*)c.ybuf, c.epart,
                           c.cnt);
}

static void launch_f64_items(const LaunchCtx& c, const int4* items, int n) {
    // FP64 FFTs of complex128 input, or of complex64 input widened on load
    auto k64 = c.in_fp64 ? syndrome_kernel<double, kFftPointsF64, double> : syndrome_kernel<double, kFftPointsF64, float>;
    if (n)
        hipLaunchKernelGGL(k64, dim3(n), dim3(kBlock), 0, c.stream, c.sigs, c.io, items, c.shifts,
                           (const double2*)c.twiddle, c.tw_log2, (double2*)c.synd, (double2*)c.ybuf, c.epart, c.cnt);
}

hipError_t launch_syndromes(const LaunchCtx& c, int part) {
    if (part != 1) {
        // the late items: general mode's random-shift lines
        if (c.fp64) {
            launch_f64_items(c, c.synd_late_items, c.n_synd_late_items);
        } else {
            launch_f32_items<kFftPointsF32Small>(c, c.synd_late_small_items, c.n_synd_late_small_items);
            launch_f32_items<kFftPointsF32>(c, c.synd_late_items, c.n_synd_late_items);
        }
        if (part == 2) return hipGetLastError();
    }
    if (c.fp64) {
        launch_f64_items(c, c.synd_items, c.n_synd_items);
        launch_f64_items(c, c.synd2_items, c.n_synd2_items);
        if (c.n_line_items)
            hipLaunchKernelGGL(line_energy_kernel<double>, dim3(c.n_line_items), dim3(kBlock), 0, c.stream, c.sigs,
                               c.line_items, (const double2*)c.synd, c.epart);
    } else {
        launch_pairs(c);
        launch_f32_items<kFftPointsF32Small>(c, c.synd_small_items, c.n_synd_small_items);
        launch_f32_items<kFftPointsF32>(c, c.synd_items, c.n_synd_items);
        launch_f32_items<kFftPointsF32>(c, c.synd2_items, c.n_synd2_items);
        if (c.n_line_items)
            hipLaunchKernelGGL(line_energy_kernel<float>, dim3(c.n_line_items), dim3(kBlock), 0, c.stream, c.sigs,
                               c.line_items, (const float2*)c.synd, c.epart);
    }
    return hipGetLastError();
}

}  // namespace sft
