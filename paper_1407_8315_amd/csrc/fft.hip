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
        // scale by d, store shift-major, per-line energy (FP64, fixed-order tree)
        V* out = synd + sg.synd_off + ((int64_t)line0 << log2m);
        for (int line = 0; line < nl; ++line) {
            double acc = 0.0;
            for (int k = threadIdx.x; k < len; k += kBlock) {
                V v = buf[(line << log2m) + k];
                v.x *= dscale;
                v.y *= dscale;
                out[((int64_t)line << log2m) + k] = v;
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
            synd[sg.synd_off + ((int64_t)l << log2m) + k2 + ((int64_t)k1 << log2m2)] = v;
        }
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
    const typename C2<T>::type* row = synd + sg.synd_off + ((int64_t)it.y << sg.log2m);
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < sg.m; k += kBlock) {
        auto v = row[k];
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

hipError_t launch_syndromes(const LaunchCtx& c) {
    if (c.fp64) {
        // FP64 FFTs of complex128 input, or of complex64 input widened on load
        auto k64 = c.in_fp64 ? syndrome_kernel<double, kFftPointsF64, double> : syndrome_kernel<double, kFftPointsF64, float>;
        if (c.n_synd_items)
            hipLaunchKernelGGL(k64, dim3(c.n_synd_items), dim3(kBlock), 0, c.stream, c.sigs, c.io, c.synd_items,
                               c.shifts, (const double2*)c.twiddle, c.tw_log2, (double2*)c.synd, (double2*)c.ybuf,
                               c.epart, c.cnt);
        if (c.n_synd2_items)
            hipLaunchKernelGGL(k64, dim3(c.n_synd2_items), dim3(kBlock), 0, c.stream, c.sigs, c.io, c.synd2_items,
                               c.shifts, (const double2*)c.twiddle, c.tw_log2, (double2*)c.synd, (double2*)c.ybuf,
                               c.epart, c.cnt);
        if (c.n_line_items)
            hipLaunchKernelGGL(line_energy_kernel<double>, dim3(c.n_line_items), dim3(kBlock), 0, c.stream, c.sigs,
                               c.line_items, (const double2*)c.synd, c.epart);
    } else {
        if (c.n_synd_small_items)
            hipLaunchKernelGGL((syndrome_kernel<float, kFftPointsF32Small, float>), dim3(c.n_synd_small_items), dim3(kBlock), 0,
                               c.stream, c.sigs, c.io, c.synd_small_items, c.shifts, (const float2*)c.twiddle,
                               c.tw_log2, (float2*)c.synd, (float2*)c.ybuf, c.epart, c.cnt);
        if (c.n_synd_items)
            hipLaunchKernelGGL((syndrome_kernel<float, kFftPointsF32, float>), dim3(c.n_synd_items), dim3(kBlock), 0, c.stream,
                               c.sigs, c.io, c.synd_items, c.shifts, (const float2*)c.twiddle, c.tw_log2,
                               (float2*)c.synd, (float2*)c.ybuf, c.epart, c.cnt);
        if (c.n_synd2_items)
            hipLaunchKernelGGL((syndrome_kernel<float, kFftPointsF32, float>), dim3(c.n_synd2_items), dim3(kBlock), 0,
                               c.stream, c.sigs, c.io, c.synd2_items, c.shifts, (const float2*)c.twiddle, c.tw_log2,
                               (float2*)c.synd, (float2*)c.ybuf, c.epart, c.cnt);
        if (c.n_line_items)
            hipLaunchKernelGGL(line_energy_kernel<float>, dim3(c.n_line_items), dim3(kBlock), 0, c.stream, c.sigs,
                               c.line_items, (const float2*)c.synd, c.epart);
    }
    return hipGetLastError();
}

}  // namespace sft
