// Learned order predictor: a small MLP that maps an active bin's syndromes to
// its number of aliased frequencies (0..4), replacing the rank test of the
// order estimate; the rank test stays as the fallback and the residual check
// as the judge.  (A project addition; its analogue in the paper is the order
// estimate of Pruning Step 1, Sec. III-C.)
//
// Network 32 -> 128 -> 128 -> 5 with GELU, BF16 weights, FP32 accumulation on
// gfx950's v_mfma_f32_16x16x32_bf16 (v_mfma_f32_16x16x16_bf16 for the one
// product with 16-long sums, dZ3 W3).  A block holds 64 rows (bins) in LDS; each of its
// 4 waves owns 16 rows in the forward pass and in the input-side backward pass;
// weight gradients reduce over the block's rows with MFMA and are added to a
// global FP32 buffer.  Adam updates FP32 master weights and refreshes the BF16
// copies.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "algebra.h"
#include "plan_host.h"

namespace sft {

constexpr int kNF = 32, kNH = 128, kNC = 5, kNCp = 16;
constexpr int kOffW1 = 0, kOffB1 = 4096, kOffW2 = 4224, kOffB2 = 20608, kOffW3 = 20736, kOffB3 = 21376;
constexpr int kNParams = 21381;
// padded LDS row strides (bf16 / float elements); rows of X and H start on
// 16-byte boundaries for the 8-element operand loads
constexpr int kLdX = 40, kLdH = 136, kLdC = 20;
constexpr int kRows = 64;                          // rows per block tile
// BF16 weight image (same padded layout in global memory and LDS)
constexpr int kW1Elems = kNH * kLdX, kW2Elems = kNH * kLdH, kW3Elems = kNCp * kLdH;
constexpr int kWElems = kW1Elems + kW2Elems + kW3Elems;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__host__ __device__ inline bf16 to_bf16(float f) {
    union {
        float f;
        unsigned u;
    } v;
    v.f = f;
    unsigned u = v.u;
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (bf16)(u >> 16);
}
__device__ inline float from_bf16(bf16 h) { return __uint_as_float(((unsigned)h) << 16); }
// gelu(x) = x Phi(x) with Phi(x) = (1 + erf(x / sqrt 2)) / 2.  erf by
// Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7 on the whole line, odd
// extension): erf(u) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-u^2},
// t = 1 / (1 + p u), u >= 0; far below the BF16 rounding of the activations,
// and lighter on registers than the library erf.  e^{-u^2} = e^{-x^2/2} is
// shared with the density in the derivative.
struct PhiPdf {
    float cdf, pdf;
};
__device__ inline PhiPdf phi_pdf(float x) {
    const float u = fabsf(x) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * u);
    const float g = __expf(-u * u);
    const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
    const float erf_u = 1.0f - poly * g;
    return PhiPdf{0.5f * (1.0f + copysignf(erf_u, x)), g * 0.39894228040143268f};
}
__device__ inline float gelu(float x) { return x * phi_pdf(x).cdf; }
__device__ inline float gelu_grad(float x) {
    const PhiPdf q = phi_pdf(x);
    return q.cdf + x * q.pdf;
}
// D (16 x 16, FP32) += A B over K = 16 or 32: lane l supplies row l % 16 of
// A and column l % 16 of B at the K positions of its lane group l / 16 (4 or
// 8 consecutive ones, the same for A and B), and holds D[4 (l / 16) + j][l % 16].
__device__ inline v4f mfma16(v4s a, v4s b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ inline v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ inline v4s ld4(const bf16* p) { return *reinterpret_cast<const v4s*>(p); }
__device__ inline v8s ld8(const bf16* p) { return *reinterpret_cast<const v8s*>(p); }
__device__ inline v8s gather8(const bf16* p, int stride) {
    v8s r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (short)p[i * stride];
    return r;
}
__device__ inline v4s gather4(const bf16* p, int stride) {
    v4s r;
    r.x = (short)p[0];
    r.y = (short)p[stride];
    r.z = (short)p[2 * stride];
    r.w = (short)p[3 * stride];
    return r;
}

struct alignas(16) WeightsLds {
    bf16 w[kWElems];                   // W1 [128][40], W2 [128][136], W3 [16][136]
    float b1[kNH], b2[kNH], b3[kNCp];
};

// Copy the BF16 image and the FP32 biases into LDS (whole block).
__device__ inline void load_weights(WeightsLds& W, const bf16* __restrict__ wimg, const float* __restrict__ theta) {
    const uint4* src = reinterpret_cast<const uint4*>(wimg);
    uint4* dst = reinterpret_cast<uint4*>(W.w);
    for (int i = threadIdx.x; i < kWElems / 8; i += blockDim.x) dst[i] = src[i];
    for (int i = threadIdx.x; i < kNH; i += blockDim.x) {
        W.b1[i] = theta[kOffB1 + i];
        W.b2[i] = theta[kOffB2 + i];
    }
    for (int i = threadIdx.x; i < kNCp; i += blockDim.x) W.b3[i] = i < kNC ? theta[kOffB3 + i] : 0.0f;
}

// Forward pass of the wave's 16 rows (r0 .. r0+15): H1, H2 (BF16, LDS) and the
// pre-activations Z1, Z2 (FP32, registers, MFMA output layout: element j of
// tile t of lane l is row r0 + 4 (l / 16) + j, column 16 t + l % 16); returns
// the logits tile (columns 0..15, valid 0..4).
struct Fwd {
    v4f z1[8], z2[8], z3;
};
__device__ inline void forward_rows(const WeightsLds& W, const bf16* X, bf16* H1, bf16* H2, int r0, Fwd& f) {
    const int l = __lane_id(), li = l & 15, lq = l >> 4;
    const bf16* w1 = W.w;
    const bf16* w2 = W.w + kW1Elems;
    const bf16* w3 = W.w + kW1Elems + kW2Elems;
#pragma unroll
    for (int t = 0; t < 8; ++t) f.z1[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNF / 32; ++kk) {
        v8s a = ld8(X + (r0 + li) * kLdX + kk * 32 + lq * 8);
#pragma unroll
        for (int t = 0; t < 8; ++t) f.z1[t] = mfma32(a, ld8(w1 + (t * 16 + li) * kLdX + kk * 32 + lq * 8), f.z1[t]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float z = f.z1[t][j] + W.b1[t * 16 + li];
            f.z1[t][j] = z;
            H1[(r0 + lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(gelu(z));
        }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) f.z2[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNH / 32; ++kk) {
        v8s a = ld8(H1 + (r0 + li) * kLdH + kk * 32 + lq * 8);
#pragma unroll
        for (int t = 0; t < 8; ++t) f.z2[t] = mfma32(a, ld8(w2 + (t * 16 + li) * kLdH + kk * 32 + lq * 8), f.z2[t]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float z = f.z2[t][j] + W.b2[t * 16 + li];
            f.z2[t][j] = z;
            H2[(r0 + lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(gelu(z));
        }
    __syncthreads();
    f.z3 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNH / 32; ++kk)
        f.z3 = mfma32(ld8(H2 + (r0 + li) * kLdH + kk * 32 + lq * 8), ld8(w3 + li * kLdH + kk * 32 + lq * 8), f.z3);
#pragma unroll
    for (int j = 0; j < 4; ++j) f.z3[j] += W.b3[li];
}

// Features of bin k of signal sg (see the module comment of the reference
// network), from its 8 raw syndromes, in FP32 (they are rounded to BF16 for
// the network; the de-rotation phase (k l mod N) / N is reduced exactly).
template <typename V>
__device__ inline void bin_features(const V* __restrict__ synd, const SigDev& sg, int64_t k, float eref, float* f) {
    float2 mt[8];
    float e = 0.0f;
#pragma unroll
    for (int l = 0; l < 8; ++l) {
        const auto v = synd[synd_at(sg, l, k)];
        const int64_t q = (k * l) & (sg.n - 1);
        float sn, cs;
        sincospif((float)(2.0 * (double)q / (double)sg.n), &sn, &cs);
        const float vx = (float)v.x, vy = (float)v.y;
        mt[l] = float2{cs * vx + sn * vy, cs * vy - sn * vx};   // e^{-i 2 pi q / N} m_l
        e += mt[l].x * mt[l].x + mt[l].y * mt[l].y;
    }
    const float rms = sqrtf(e / 8.0f);
    const float a0 = sqrtf(mt[0].x * mt[0].x + mt[0].y * mt[0].y);
    const float px = a0 > 0.0f ? mt[0].x / a0 : 1.0f, py = a0 > 0.0f ? -mt[0].y / a0 : 0.0f;
    const float ir = 1.0f / rms;
#pragma unroll
    for (int l = 0; l < 8; ++l) {
        f[2 * l] = (mt[l].x * px - mt[l].y * py) * ir;
        f[2 * l + 1] = (mt[l].x * py + mt[l].y * px) * ir;
        f[16 + l] = sqrtf(mt[l].x * mt[l].x + mt[l].y * mt[l].y) * ir;
    }
    f[24] = logf(e / eref);
#pragma unroll
    for (int i = 25; i < kNF; ++i) f[i] = 0.0f;
}

__device__ inline float mean_bin_energy(const LaunchCtx& c, const SigDev& sg) {
    double eref = 0.0;
#pragma unroll
    for (int l = 0; l < 8; ++l) eref += c.epart[sg.epart_off + l];
    return (float)(eref / (double)sg.m);
}

template <typename T>
struct VT;
template <>
struct VT<float> {
    using type = float2;
};
template <>
struct VT<double> {
    using type = double2;
};

// Orders the LDS traffic of one wave (its own rows only: no block barrier).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Logits of the 16 rows X[r0 .. r0+15] by one wave, with Hw the wave's own
// 16-row activation buffer (reused by both hidden layers).  Returns the
// logits tile in the MFMA output layout (row 4 (lane / 16) + j, column lane % 16).
__device__ inline v4f infer_rows(const WeightsLds& W, const bf16* X, int r0, bf16* Hw) {
    const int l = __lane_id(), li = l & 15, lq = l >> 4;
    const bf16* w1 = W.w;
    const bf16* w2 = W.w + kW1Elems;
    const bf16* w3 = W.w + kW1Elems + kW2Elems;
    v4f z[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) z[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNF / 32; ++kk) {
        v8s a = ld8(X + (r0 + li) * kLdX + kk * 32 + lq * 8);
#pragma unroll
        for (int t = 0; t < 8; ++t) z[t] = mfma32(a, ld8(w1 + (t * 16 + li) * kLdX + kk * 32 + lq * 8), z[t]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) Hw[(lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(gelu(z[t][j] + W.b1[t * 16 + li]));
    wave_sync();
    v8s a[kNH / 32];
#pragma unroll
    for (int kk = 0; kk < kNH / 32; ++kk) a[kk] = ld8(Hw + li * kLdH + kk * 32 + lq * 8);
    wave_sync();
#pragma unroll
    for (int t = 0; t < 8; ++t) z[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNH / 32; ++kk)
#pragma unroll
        for (int t = 0; t < 8; ++t) z[t] = mfma32(a[kk], ld8(w2 + (t * 16 + li) * kLdH + kk * 32 + lq * 8), z[t]);
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) Hw[(lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(gelu(z[t][j] + W.b2[t * 16 + li]));
    wave_sync();
    v4f z3 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kNH / 32; ++kk)
        z3 = mfma32(ld8(Hw + li * kLdH + kk * 32 + lq * 8), ld8(w3 + li * kLdH + kk * 32 + lq * 8), z3);
    wave_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) z3[j] += W.b3[li];
    return z3;
}

constexpr int kInferWaves = 8;
constexpr int kInferTile = 64 * kInferWaves;   // rows per block trip: one per thread

// Learned orders for the bins the rank-one certificate left pending (exact
// mode, L = 4): each thread builds the features of one bin, each wave runs
// the network on 64 rows (4 MFMA row tiles), and the bin is queued for round
// 0 at its predicted order.  A prediction of 0 (outside 1..L) sends the bin
// to the rank test: in plans without general-mode signals that is the rest
// kernel's own (set 1, slot 0, step 0), otherwise the SVD pass before round 0.
// Blocks with no rows return before loading the weights.
template <typename T>
__global__ __launch_bounds__(kInferTile) void infer_kernel(LaunchCtx c, const bf16* __restrict__ wimg,
                                                           const float* __restrict__ theta) {
    __shared__ WeightsLds W;
    __shared__ __attribute__((aligned(16))) bf16 X[kInferTile * kLdX];
    __shared__ __attribute__((aligned(16))) bf16 H[kInferWaves * 16 * kLdH];
    __shared__ float Zs[kInferWaves * 16 * 8];
    __shared__ signed char pred[kInferTile];
    __shared__ BlockQueues bq;
    const int total = c.work->q[kQPending];
    if ((int64_t)blockIdx.x * kInferTile >= total) return;   // the whole block: no barrier is left waiting
    load_weights(W, wimg, theta);
    const int2* in = c.qlist + (int64_t)kQPending * c.list_cap;
    const typename VT<T>::type* synd = (const typename VT<T>::type*)c.synd;
    const int w = threadIdx.x >> 6, lane = __lane_id();
    for (int base = blockIdx.x * kInferTile; base < total; base += gridDim.x * kInferTile) {
        bq.reset();
        const int item = base + threadIdx.x;
        int s = -1;
        int64_t k = 0;
        float f[kNF];
#pragma unroll
        for (int i = 0; i < kNF; ++i) f[i] = 0.0f;
        if (item < total) {
            const int2 en = in[item];
            s = en.x;
            k = code_k(en.y);
            const SigDev& sg = c.sigs[s];
            bin_features(synd, sg, k, mean_bin_energy(c, sg), f);
        }
        uint2* xr = reinterpret_cast<uint2*>(X + threadIdx.x * kLdX);
#pragma unroll
        for (int i = 0; i < kNF / 4; ++i)
            xr[i] = uint2{(unsigned)to_bf16(f[4 * i]) | ((unsigned)to_bf16(f[4 * i + 1]) << 16),
                          (unsigned)to_bf16(f[4 * i + 2]) | ((unsigned)to_bf16(f[4 * i + 3]) << 16)};
        __syncthreads();
        bf16* Hw = H + w * 16 * kLdH;
        float* Zw = Zs + w * 16 * 8;
        for (int sub = 0; sub < 4; ++sub) {
            const int r0 = w * 64 + sub * 16;
            const v4f z3 = infer_rows(W, X, r0, Hw);
            const int li = lane & 15, lq = lane >> 4;
            if (li < kNC)
#pragma unroll
                for (int j = 0; j < 4; ++j) Zw[(lq * 4 + j) * 8 + li] = z3[j];
            wave_sync();
            if (lane < 16) {
                int best = 0;
                float bv = Zw[lane * 8];
                for (int cl = 1; cl < kNC; ++cl)
                    if (Zw[lane * 8 + cl] > bv) {
                        bv = Zw[lane * 8 + cl];
                        best = cl;
                    }
                pred[r0 + lane] = (signed char)best;
            }
            wave_sync();
        }
        __syncthreads();
        int q = -1;
        int2 ent{0, 0};
        if (s >= 0) {
            int ap = pred[threadIdx.x];
            if (ap < 1 || ap > c.sigs[s].L) ap = 0;
            q = (ap == 0 && c.n_general == 0) ? q_round(1, 0) : q_round(0, ap);
            ent = int2{s, pack_code(k, 0, ap, 0)};
        }
        const int slot = bq.reserve(q);
        bq.commit(c.work, c.active_list, c.qlist, c.list_cap, q, slot, ent);
    }
}

// Features of the active bins of a single-signal plan, for training data.
template <typename T>
__global__ __launch_bounds__(256) void features_kernel(LaunchCtx c, float* __restrict__ feat, int64_t* __restrict__ bins,
                                                       int64_t cap) {
    const int total = c.work->n_active;
    const typename VT<T>::type* synd = (const typename VT<T>::type*)c.synd;
    for (int item = blockIdx.x * blockDim.x + threadIdx.x; item < total; item += gridDim.x * blockDim.x) {
        if (item >= cap) continue;
        const int2 en = c.active_list[item];
        const SigDev& sg = c.sigs[en.x];
        const int64_t k = code_k(en.y);
        float f[kNF];
        bin_features(synd, sg, k, mean_bin_energy(c, sg), f);
        for (int i = 0; i < kNF; ++i) feat[(int64_t)item * kNF + i] = f[i];
        bins[item] = k;
    }
}

// Logits of given feature rows (forward pass only).
__global__ __launch_bounds__(256) void forward_kernel(const float* __restrict__ feat, int rows,
                                                      const bf16* __restrict__ wimg, const float* __restrict__ theta,
                                                      float* __restrict__ logits) {
    __shared__ WeightsLds W;
    __shared__ __attribute__((aligned(16))) bf16 X[kRows * kLdX];
    __shared__ __attribute__((aligned(16))) bf16 H1[kRows * kLdH];
    __shared__ __attribute__((aligned(16))) bf16 H2[kRows * kLdH];
    load_weights(W, wimg, theta);
    const int w = threadIdx.x >> 6;
    for (int base = blockIdx.x * kRows; base < rows; base += gridDim.x * kRows) {
        __syncthreads();
        for (int i = threadIdx.x; i < kRows * kNF; i += blockDim.x) {
            const int r = i / kNF, col = i % kNF;
            X[r * kLdX + col] = (base + r < rows) ? to_bf16(feat[(int64_t)(base + r) * kNF + col]) : (bf16)0;
        }
        __syncthreads();
        Fwd fw;
        forward_rows(W, X, H1, H2, w * 16, fw);
        const int l = __lane_id(), li = l & 15, lq = l >> 4;
        if (li < kNC)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = base + w * 16 + lq * 4 + j;
                if (r < rows) logits[(int64_t)r * kNC + li] = fw.z3[j];
            }
    }
}

// Gradient of the mean cross-entropy over `rows` labelled feature rows, added
// into grad (FP32 [kNParams]); the loss is added into *loss.
__global__ __launch_bounds__(256) void grad_kernel(const float* __restrict__ feat, const int* __restrict__ labels,
                                                   int rows, const bf16* __restrict__ wimg,
                                                   const float* __restrict__ theta, float* __restrict__ grad,
                                                   float* __restrict__ loss) {
    __shared__ WeightsLds W;
    __shared__ __attribute__((aligned(16))) bf16 X[kRows * kLdX];
    __shared__ __attribute__((aligned(16))) bf16 H1[kRows * kLdH];
    __shared__ __attribute__((aligned(16))) bf16 H2[kRows * kLdH];
    __shared__ __attribute__((aligned(16))) bf16 D1[kRows * kLdH];   // dZ1
    __shared__ __attribute__((aligned(16))) bf16 D2[kRows * kLdH];   // dZ2
    __shared__ __attribute__((aligned(16))) bf16 D3[kRows * kLdC];   // dZ3 (16 columns used)
    __shared__ float Z[kRows * kLdC];   // logits, then dZ3 in FP32
    __shared__ float red[256];
    load_weights(W, wimg, theta);
    const bf16* w2 = W.w + kW1Elems;
    const bf16* w3 = W.w + kW1Elems + kW2Elems;
    const int w = threadIdx.x >> 6;
    const int l = __lane_id(), li = l & 15, lq = l >> 4;
    const float inv_n = 1.0f / (float)rows;
    for (int base = blockIdx.x * kRows; base < rows; base += gridDim.x * kRows) {
        __syncthreads();
        for (int i = threadIdx.x; i < kRows * kNF; i += blockDim.x) {
            const int r = i / kNF, col = i % kNF;
            X[r * kLdX + col] = (base + r < rows) ? to_bf16(feat[(int64_t)(base + r) * kNF + col]) : (bf16)0;
        }
        __syncthreads();
        Fwd fw;
        forward_rows(W, X, H1, H2, w * 16, fw);
#pragma unroll
        for (int j = 0; j < 4; ++j) Z[(w * 16 + lq * 4 + j) * kLdC + li] = fw.z3[j];
        __syncthreads();
        // softmax, loss and dZ3 = (p - onehot) / n per row; padding rows get 0
        float my_loss = 0.0f;
        if (threadIdx.x < kRows) {
            const int r = threadIdx.x;
            const bool valid = base + r < rows;
            float zmax = Z[r * kLdC];
            for (int cl = 1; cl < kNC; ++cl) zmax = fmaxf(zmax, Z[r * kLdC + cl]);
            float p[kNC], sum = 0.0f;
            for (int cl = 0; cl < kNC; ++cl) {
                p[cl] = expf(Z[r * kLdC + cl] - zmax);
                sum += p[cl];
            }
            const int y = valid ? labels[base + r] : 0;
            for (int cl = 0; cl < kNCp; ++cl) {
                float g = 0.0f;
                if (valid && cl < kNC) g = (p[cl] / sum - (cl == y ? 1.0f : 0.0f)) * inv_n;
                Z[r * kLdC + cl] = g;
                D3[r * kLdC + cl] = to_bf16(g);
            }
            if (valid) my_loss = -logf(p[y] / sum);
        }
        red[threadIdx.x] = my_loss;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicAdd(loss, red[0] * inv_n);
        // dH2 = dZ3 W3 (own rows), dZ2 = dH2 * gelu'(Z2)
        {
            v4f acc[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
            v4s a = ld4(D3 + (w * 16 + li) * kLdC + lq * 4);
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = mfma16(a, gather4(w3 + (lq * 4) * kLdH + t * 16 + li, kLdH), acc[t]);
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    D2[(w * 16 + lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(acc[t][j] * gelu_grad(fw.z2[t][j]));
        }
        __syncthreads();
        // dH1 = dZ2 W2 (own rows), dZ1 = dH1 * gelu'(Z1)
        {
            v4f acc[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kNH / 32; ++kk) {
                v8s a = ld8(D2 + (w * 16 + li) * kLdH + kk * 32 + lq * 8);
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    acc[t] = mfma32(a, gather8(w2 + (kk * 32 + lq * 8) * kLdH + t * 16 + li, kLdH), acc[t]);
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    D1[(w * 16 + lq * 4 + j) * kLdH + t * 16 + li] = to_bf16(acc[t][j] * gelu_grad(fw.z1[t][j]));
        }
        __syncthreads();
        // weight gradients, reduced over the 64 rows: dW = dZ^T H (MFMA, K = rows)
        // dW2 [128][128]: 64 tiles, 16 per wave
        for (int tile = w; tile < 64; tile += 4) {
            const int tm = tile >> 3, tn = tile & 7;
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kRows / 32; ++kk) {
                v8s a = gather8(D2 + (kk * 32 + lq * 8) * kLdH + tm * 16 + li, kLdH);
                v8s b = gather8(H1 + (kk * 32 + lq * 8) * kLdH + tn * 16 + li, kLdH);
                acc = mfma32(a, b, acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                atomicAdd(&grad[kOffW2 + (tm * 16 + lq * 4 + j) * kNH + tn * 16 + li], acc[j]);
        }
        // dW1 [128][32]: 16 tiles, 4 per wave
        for (int tile = w; tile < 16; tile += 4) {
            const int tm = tile >> 1, tn = tile & 1;
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kRows / 32; ++kk) {
                v8s a = gather8(D1 + (kk * 32 + lq * 8) * kLdH + tm * 16 + li, kLdH);
                v8s b = gather8(X + (kk * 32 + lq * 8) * kLdX + tn * 16 + li, kLdX);
                acc = mfma32(a, b, acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                atomicAdd(&grad[kOffW1 + (tm * 16 + lq * 4 + j) * kNF + tn * 16 + li], acc[j]);
        }
        // dW3 [5][128]: 8 tiles (rows 0..15, 5 valid), 2 per wave
        for (int tn = w; tn < 8; tn += 4) {
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kRows / 32; ++kk) {
                v8s a = gather8(D3 + (kk * 32 + lq * 8) * kLdC + li, kLdC);
                v8s b = gather8(H2 + (kk * 32 + lq * 8) * kLdH + tn * 16 + li, kLdH);
                acc = mfma32(a, b, acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (lq * 4 + j < kNC) atomicAdd(&grad[kOffW3 + (lq * 4 + j) * kNH + tn * 16 + li], acc[j]);
        }
        // bias gradients: column sums of dZ1, dZ2 (BF16 copies) and dZ3 (FP32)
        for (int col = threadIdx.x; col < 2 * kNH + kNC; col += blockDim.x) {
            float sacc = 0.0f;
            if (col < kNH) {
                for (int r = 0; r < kRows; ++r) sacc += from_bf16(D1[r * kLdH + col]);
                atomicAdd(&grad[kOffB1 + col], sacc);
            } else if (col < 2 * kNH) {
                for (int r = 0; r < kRows; ++r) sacc += from_bf16(D2[r * kLdH + col - kNH]);
                atomicAdd(&grad[kOffB2 + col - kNH], sacc);
            } else {
                for (int r = 0; r < kRows; ++r) sacc += Z[r * kLdC + col - 2 * kNH];
                atomicAdd(&grad[kOffB3 + col - 2 * kNH], sacc);
            }
        }
    }
}

__global__ void zero_kernel(float* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void count_kernel(const WorkCounters* work, int64_t* count) { *count = work->n_active; }

// Adam on the FP32 master weights; refreshes the BF16 image and clears grad.
__global__ void adam_kernel(float* __restrict__ theta, float* __restrict__ grad, float* __restrict__ m1,
                            float* __restrict__ m2, bf16* __restrict__ wimg, float lr, float b1c, float b2c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    const float g = grad[i];
    const float a = 0.9f * m1[i] + 0.1f * g;
    const float b = 0.999f * m2[i] + 0.001f * g * g;
    m1[i] = a;
    m2[i] = b;
    const float p = theta[i] - lr * (a / b1c) / (sqrtf(b / b2c) + 1e-8f);
    theta[i] = p;
    grad[i] = 0.0f;
    // position in the BF16 image
    int pos = -1;
    if (i < kOffB1) pos = (i / kNF) * kLdX + (i % kNF);
    else if (i >= kOffW2 && i < kOffB2) pos = kW1Elems + ((i - kOffW2) / kNH) * kLdH + ((i - kOffW2) % kNH);
    else if (i >= kOffW3 && i < kOffB3) pos = kW1Elems + kW2Elems + ((i - kOffW3) / kNH) * kLdH + ((i - kOffW3) % kNH);
    if (pos >= 0) wimg[pos] = to_bf16(p);
}

}  // namespace sft

using namespace sft;

struct sft_mlp_s {
    hipStream_t stream = nullptr;
    float* theta = nullptr;   // FP32 master [kNParams]
    float* grad = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    bf16* wimg = nullptr;     // BF16 image [kWElems]
    float* scratch_loss = nullptr;
    int64_t step = 0;
};

namespace {

thread_local std::string g_mlp_err;

sft_status mfail(sft_status s, const std::string& m) {
    g_mlp_err = m;
    return s;
}

#define MHIP(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return mfail(SFT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

std::vector<bf16> host_image(const std::vector<float>& th) {
    std::vector<bf16> img((size_t)kWElems, 0);
    for (int i = 0; i < kNH * kNF; ++i) img[(size_t)((i / kNF) * kLdX + i % kNF)] = to_bf16(th[(size_t)(kOffW1 + i)]);
    for (int i = 0; i < kNH * kNH; ++i)
        img[(size_t)(kW1Elems + (i / kNH) * kLdH + i % kNH)] = to_bf16(th[(size_t)(kOffW2 + i)]);
    for (int i = 0; i < kNC * kNH; ++i)
        img[(size_t)(kW1Elems + kW2Elems + (i / kNH) * kLdH + i % kNH)] = to_bf16(th[(size_t)(kOffW3 + i)]);
    return img;
}

sft_status upload(sft_mlp_t m, const std::vector<float>& th) {
    std::vector<bf16> img = host_image(th);
    MHIP(hipMemcpy(m->theta, th.data(), th.size() * sizeof(float), hipMemcpyHostToDevice));
    MHIP(hipMemcpy(m->wimg, img.data(), img.size() * sizeof(bf16), hipMemcpyHostToDevice));
    MHIP(hipMemset(m->grad, 0, kNParams * sizeof(float)));
    MHIP(hipMemset(m->m1, 0, kNParams * sizeof(float)));
    MHIP(hipMemset(m->m2, 0, kNParams * sizeof(float)));
    m->step = 0;
    return SFT_OK;
}

int grid_for(int64_t rows) {
    int64_t b = (rows + kRows - 1) / kRows;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace

// Learned mode hook: run the predictor over the active list (after the
// activity pass, before the decoder).
sft_status sft_mlp_launch_infer(sft_mlp_t m, const LaunchCtx& c) {
    if (!m) return SFT_OK;
    // one block of kInferTile rows per CU at a time (the block holds ~124 KiB of LDS)
    const int grid = std::max(1, std::min(c.n_work_blocks, 512));
    if (c.fp64)
        hipLaunchKernelGGL(infer_kernel<double>, dim3(grid), dim3(kInferTile), 0, c.stream, c, m->wimg, m->theta);
    else
        hipLaunchKernelGGL(infer_kernel<float>, dim3(grid), dim3(kInferTile), 0, c.stream, c, m->wimg, m->theta);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFT_OK : mfail(SFT_E_DEVICE, hipGetErrorString(e));
}

sft_status sft_features_enqueue(const LaunchCtx& c, float* feat, int64_t* bins, int64_t cap, int64_t* count) {
    hipLaunchKernelGGL(count_kernel, dim3(1), dim3(1), 0, c.stream, c.work, count);
    if (c.fp64)
        hipLaunchKernelGGL(features_kernel<double>, dim3(c.n_work_blocks), dim3(256), 0, c.stream, c, feat, bins, cap);
    else
        hipLaunchKernelGGL(features_kernel<float>, dim3(c.n_work_blocks), dim3(256), 0, c.stream, c, feat, bins, cap);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFT_OK : mfail(SFT_E_DEVICE, hipGetErrorString(e));
}

hipStream_t sft_mlp_stream(sft_mlp_t m) { return m->stream; }

extern "C" {

sft_status sft_mlp_create(sft_mlp_t* out, uint64_t seed, void* hip_stream) {
    if (!out) return mfail(SFT_E_INVALID, "out is NULL");
    *out = nullptr;
    sft_mlp_s* m = new sft_mlp_s();
    m->stream = (hipStream_t)hip_stream;
    bool ok = hipMalloc(&m->theta, kNParams * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->grad, kNParams * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->m1, kNParams * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->m2, kNParams * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->wimg, kWElems * sizeof(bf16)) == hipSuccess &&
              hipMalloc(&m->scratch_loss, sizeof(float)) == hipSuccess;
    if (!ok) {
        sft_mlp_destroy(m);
        return mfail(SFT_E_NOMEM, "hipMalloc failed");
    }
    // uniform initialisation, bound sqrt(6 / fan_in) (He uniform), biases 0
    std::vector<float> th((size_t)kNParams, 0.0f);
    uint64_t st = seed ^ 0x6a09e667f3bcc909ull;
    auto next = [&st]() {
        uint64_t z = (st += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int count, int fan_in) {
        const double bound = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < count; ++i) th[(size_t)(off + i)] = (float)((2.0 * next() - 1.0) * bound);
    };
    fill(kOffW1, kNH * kNF, kNF);
    fill(kOffW2, kNH * kNH, kNH);
    fill(kOffW3, kNC * kNH, kNH);
    sft_status s = upload(m, th);
    if (s != SFT_OK) {
        sft_mlp_destroy(m);
        return s;
    }
    *out = m;
    return SFT_OK;
}

void sft_mlp_destroy(sft_mlp_t m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    if (m->theta) (void)hipFree(m->theta);
    if (m->grad) (void)hipFree(m->grad);
    if (m->m1) (void)hipFree(m->m1);
    if (m->m2) (void)hipFree(m->m2);
    if (m->wimg) (void)hipFree(m->wimg);
    if (m->scratch_loss) (void)hipFree(m->scratch_loss);
    delete m;
}

sft_status sft_mlp_get_params(sft_mlp_t m, float* host, int64_t n) {
    if (!m || !host) return mfail(SFT_E_INVALID, "NULL argument");
    if (n != kNParams) return mfail(SFT_E_INVALID, "need exactly SFT_MLP_PARAMS values");
    MHIP(hipStreamSynchronize(m->stream));
    MHIP(hipMemcpy(host, m->theta, kNParams * sizeof(float), hipMemcpyDeviceToHost));
    return SFT_OK;
}

sft_status sft_mlp_set_params(sft_mlp_t m, const float* host, int64_t n) {
    if (!m || !host) return mfail(SFT_E_INVALID, "NULL argument");
    if (n != kNParams) return mfail(SFT_E_INVALID, "need exactly SFT_MLP_PARAMS values");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return mfail(SFT_E_INVALID, "non-finite parameter");
    MHIP(hipStreamSynchronize(m->stream));
    return upload(m, std::vector<float>(host, host + n));
}

sft_status sft_mlp_forward(sft_mlp_t m, const float* feat_dev, int64_t rows, float* logits_dev) {
    if (!m || !feat_dev || !logits_dev || rows < 0) return mfail(SFT_E_INVALID, "bad argument");
    if (rows > (int64_t(1) << 30)) return mfail(SFT_E_UNSUPPORTED, "too many rows");
    if (rows == 0) return SFT_OK;
    hipLaunchKernelGGL(forward_kernel, dim3(grid_for(rows)), dim3(256), 0, m->stream, feat_dev, (int)rows, m->wimg,
                       m->theta, logits_dev);
    MHIP(hipGetLastError());
    return SFT_OK;
}

sft_status sft_mlp_grad(sft_mlp_t m, const float* feat_dev, const int32_t* labels_dev, int64_t rows, float* grad_dev,
                        float* loss_dev) {
    if (!m || !feat_dev || !labels_dev || !grad_dev || !loss_dev || rows < 1)
        return mfail(SFT_E_INVALID, "bad argument");
    if (rows > (int64_t(1) << 30)) return mfail(SFT_E_UNSUPPORTED, "too many rows");
    hipLaunchKernelGGL(zero_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, m->stream, grad_dev, kNParams);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, m->stream, loss_dev, 1);
    hipLaunchKernelGGL(grad_kernel, dim3(grid_for(rows)), dim3(256), 0, m->stream, feat_dev, labels_dev, (int)rows,
                       m->wimg, m->theta, grad_dev, loss_dev);
    MHIP(hipGetLastError());
    return SFT_OK;
}

sft_status sft_mlp_train_step(sft_mlp_t m, const float* feat_dev, const int32_t* labels_dev, int64_t rows, float lr,
                              float* loss_dev) {
    if (!m || !feat_dev || !labels_dev || rows < 1 || !(lr > 0.0f)) return mfail(SFT_E_INVALID, "bad argument");
    if (rows > (int64_t(1) << 30)) return mfail(SFT_E_UNSUPPORTED, "too many rows");
    float* loss = loss_dev ? loss_dev : m->scratch_loss;
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, m->stream, loss, 1);
    hipLaunchKernelGGL(grad_kernel, dim3(grid_for(rows)), dim3(256), 0, m->stream, feat_dev, labels_dev, (int)rows,
                       m->wimg, m->theta, m->grad, loss);
    MHIP(hipGetLastError());
    m->step += 1;
    const float b1c = 1.0f - std::pow(0.9f, (float)m->step);
    const float b2c = 1.0f - std::pow(0.999f, (float)m->step);
    hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, m->stream, m->theta, m->grad, m->m1,
                       m->m2, m->wimg, lr, b1c, b2c);
    MHIP(hipGetLastError());
    return SFT_OK;
}

const char* sft_mlp_last_error(void) { return g_mlp_err.c_str(); }

}  // extern "C"
