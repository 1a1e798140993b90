// sph_mlp.hip -- the learned warm-start MLP on gfx950 matrix cores.
//
// Network per particle: five dimensionless features -> 64 -> 64 -> 1, ReLU;
// bf16 weights and activations (round to nearest even), FP32 accumulation,
// FP32 biases.  Parameter vector (FP32 masters, 4620 floats):
//   W1[64][5] b1[64] W2[64][64] b2[64] w3[64] b3 in_shift[5] in_scale[5] out_scale
//
// A wave processes 32 samples per tile with v_mfma_f32_32x32x8_bf16.  Every
// layer is computed transposed (hidden units as rows, samples as columns):
// then the D registers of one layer, lane = sample + 32*half, register r =
// row 8*(r/4) + 4*half + r%4, are exactly the B operand of the next layer's
// 8-row k-chunks (registers 4c..4c+3 of chunk c), so activations never leave
// registers in the forward pass.  Training adds the backward product through
// W2^T (same trick), the weight-gradient GEMM dZ2^T H1 over the samples of a
// tile (operands transposed through LDS), and FP32 row sums for the small
// gradients; per-workgroup partials are summed in a fixed order, no float
// atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstddef>

#include "sph_internal.h"

namespace sph {
namespace {

constexpr int H = 64;
constexpr int NF = 5;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * NF, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H, OFF_SHIFT = OFF_B3 + 1, OFF_SCALE = OFF_SHIFT + NF, OFF_OUT = OFF_SCALE + NF,
              NPARAM = OFF_OUT + 1;
static_assert(NPARAM == 4620, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ReLU as one integer max on the bit pattern: every float with the sign bit
// set (negatives, -0) becomes +0, the rest is unchanged (fmaxf costs a second,
// canonicalising max per value)
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ f32x16 mfma(bf16x4 a, bf16x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// D-layout row of register r in a 32-row tile for a lane in half h
__device__ __forceinline__ int drow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ bf16x4 pack4(const uint16_t* p) {
    bf16x4 v;
    v[0] = (short)p[0]; v[1] = (short)p[1]; v[2] = (short)p[2]; v[3] = (short)p[3];
    return v;
}

// four consecutive bf16 at an 8-byte aligned LDS address, one 64-bit read
__device__ __forceinline__ bf16x4 load4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

// Weights as bf16 in LDS: W1b[64][8] (k padded with zeros), W2b[64][64], W2t[64][64] (transposed)
struct alignas(16) WeightsLDS {
    uint16_t W1b[H * 8];
    uint16_t W2b[H * H];
    uint16_t W2t[H * H];
    float b1[H], b2[H], w3[H];     // w3 as the bf16-rounded value in FP32
    float shift[8], scale[8];
    float b3, out_scale;
};

__device__ void load_weights(WeightsLDS& W, const float* __restrict__ P, bool transposed) {
    for (int t = threadIdx.x; t < H * 8; t += blockDim.x) {
        const int j = t >> 3, k = t & 7;
        W.W1b[t] = k < NF ? to_bf16(P[OFF_W1 + j * NF + k]) : (uint16_t)0;
    }
    for (int t = threadIdx.x; t < H * H; t += blockDim.x) {
        const uint16_t b = to_bf16(P[OFF_W2 + t]);
        W.W2b[t] = b;
        if (transposed) W.W2t[(t % H) * H + t / H] = b;
    }
    for (int t = threadIdx.x; t < H; t += blockDim.x) {
        W.b1[t] = P[OFF_B1 + t];
        W.b2[t] = P[OFF_B2 + t];
        W.w3[t] = from_bf16(to_bf16(P[OFF_W3 + t]));
    }
    if (threadIdx.x < 8) {
        W.shift[threadIdx.x] = threadIdx.x < NF ? P[OFF_SHIFT + threadIdx.x] : 0.f;
        W.scale[threadIdx.x] = threadIdx.x < NF ? P[OFF_SCALE + threadIdx.x] : 0.f;
    }
    if (threadIdx.x == 0) {
        W.b3 = P[OFF_B3];
        W.out_scale = P[OFF_OUT];
    }
    __syncthreads();
}

// A operands of layers 1 and 2 for this lane (row p of each 32-row tile,
// k-chunk half h), held in registers across the tiles a wave processes.
struct AOps {
    bf16x4 w1[2];
    bf16x4 w2[2][8];
};

__device__ __forceinline__ void load_aops(const WeightsLDS& W, AOps& a) {
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        a.w1[t] = load4(&W.W1b[(32 * t + p) * 8 + 4 * h]);
#pragma unroll
        for (int b = 0; b < 8; ++b) a.w2[t][b] = load4(&W.W2b[(32 * t + p) * H + 8 * b + 4 * h]);
    }
}

// Forward of one 32-sample tile in one wave.  lane = p + 32 h.
struct Fwd {
    f32x16 z1[2], z2[2];   // pre-activations, transposed tiles (rows = hidden units)
    bf16x4 h1[2][4];       // bf16(relu(z1)) as B operands, chunk c of tile t
    float h2[2][16];       // bf16(relu(z2)) as FP32
    float z;               // output before out_scale (every lane, for its sample p)
    bf16x4 xb;             // normalised features as the layer-1 B operand
};

__device__ __forceinline__ void forward_tile(const WeightsLDS& W, const AOps& A, const float* __restrict__ feat,
                                             int64_t n, int64_t base, Fwd& f) {
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const int64_t s = base + p;
    // features 4h..4h+3 of sample p, normalised in FP32 then rounded to bf16
    uint16_t xv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = 4 * h + c;
        float v = 0.f;
        if (k < NF && s < n) {
#pragma clang fp contract(off)
            v = (feat[s * NF + k] - W.shift[k]) * W.scale[k];
        }
        xv[c] = to_bf16(v);
    }
    f.xb = pack4(xv);
    // layer 1: z1^T[j][p] = sum_k W1[j][k] x[p][k] + b1[j]
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16 c;
#pragma unroll
        for (int r = 0; r < 16; ++r) c[r] = W.b1[32 * t + drow(r, h)];
        f.z1[t] = mfma(A.w1[t], f.xb, c);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            uint16_t q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = to_bf16(relu(f.z1[t][4 * cc + u]));
            f.h1[t][cc] = pack4(q);
        }
    }
    // layer 2: z2^T[j][p] = sum_k W2[j][k] h1[p][k] + b2[j]; k-chunk b covers 8b..8b+7
    float part = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16 c;
#pragma unroll
        for (int r = 0; r < 16; ++r) c[r] = W.b2[32 * t + drow(r, h)];
#pragma unroll
        for (int b = 0; b < 8; ++b) c = mfma(A.w2[t][b], f.h1[b >> 2][b & 3], c);
        f.z2[t] = c;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float hv = from_bf16(to_bf16(relu(c[r])));
            f.h2[t][r] = hv;
            part += hv * W.w3[32 * t + drow(r, h)];
        }
    }
    // layer 3: the two halves of the wave hold complementary rows
    part += __shfl_xor(part, 32, 64);
    f.z = part + W.b3;
}

// ---------------------------------------------------------------- inference
// Inference keeps every weight and bias a lane needs in registers and runs
// layer 2 on v_mfma_f32_32x32x16_bf16 (K = 16 per instruction, twice the
// rate of the 32x32x8 form).  A lane contributes eight k values per
// operand; the contraction does not depend on which eight as long as A and
// B agree, so lane half h of chunk c takes the hidden units that the
// layer-1 D registers 8(c&1)..8(c&1)+7 of tile c>>1 already hold:
// k = 32 (c>>1) + 8 (2 (c&1) + e/4) + 4 h + e%4 for element e.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int k16(int c, int h, int e) { return 32 * (c >> 1) + 8 * (2 * (c & 1) + (e >> 2)) + 4 * h + (e & 3); }

typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// bf16(relu(x)) of z[r0..r0+7]: round pairs to bf16 (one v_cvt_pk_bf16_f32
// each), then clamp at zero as 16-bit integers (one v_pk_max_i16 per pair: a
// bf16 with the sign bit set is a negative int16, and rounding keeps the
// sign, so this equals rounding relu(x))
__device__ __forceinline__ bf16x8 relu_bf16x8(const f32x16& z, int r0) {
    u32x4 w;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const f32x2 f = {z[r0 + 2 * k], z[r0 + 2 * k + 1]};
        w[k] = __builtin_bit_cast(unsigned int, __builtin_convertvector(f, bf16x2));
    }
    i16x8 q = __builtin_bit_cast(i16x8, w);
    q = __builtin_elementwise_max(q, (i16x8)0);
    return __builtin_bit_cast(bf16x8, q);
}

struct InferRegs {
    bf16x4 w1[2];
    bf16x8 w2[2][4];
    bf16x8 w3[4];          // layer 3 as row 0 of an A operand (rows 1..31 zero)
};

// Inference operands, prepared once per parameter change by k_mlp_pack: the
// InferRegs image of every lane, dword d of lane l at word d * 64 + l (so a
// wave reads each dword with one coalesced load), then InferConst.
constexpr int kImageWords = 52;
static_assert(sizeof(InferRegs) == 4 * kImageWords, "register image");

// constants every lane needs: b1 and b2 in D-register order,
// [layer][tile t][lane half h][register r] = b[32 t + drow(r, h)], read by all
// lanes of a half at one address; the input normalisation; b3, out_scale
struct alignas(16) InferConst {
    float bperm[2][2][2][16];
    float shift[8], scale[8];
    float b3, out_scale, pad[2];
};
constexpr int kConstWords = sizeof(InferConst) / 4;
constexpr int kPackedWords = 64 * kImageWords + kConstWords;

__global__ void __launch_bounds__(64) k_mlp_pack(const float* __restrict__ P, uint32_t* __restrict__ packed) {
    const int lane = threadIdx.x, p = lane & 31, h = lane >> 5;
    InferRegs R;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * h + e;
            R.w1[t][e] = k < NF ? (short)to_bf16(P[OFF_W1 + (32 * t + p) * NF + k]) : (short)0;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int e = 0; e < 8; ++e) R.w2[t][c][e] = (__bf16)P[OFF_W2 + (32 * t + p) * H + k16(c, h, e)];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) R.w3[c][e] = p == 0 ? (__bf16)P[OFF_W3 + k16(c, h, e)] : (__bf16)0.0f;
    const uint32_t* img = reinterpret_cast<const uint32_t*>(&R);
#pragma unroll
    for (int d = 0; d < kImageWords; ++d) packed[d * 64 + lane] = img[d];
    InferConst* C = reinterpret_cast<InferConst*>(packed + 64 * kImageWords);
    for (int q = lane; q < 128; q += 64) {
        const int l = q >> 6, t = (q >> 5) & 1, hh = (q >> 4) & 1, r = q & 15;
        C->bperm[l][t][hh][r] = P[(l == 0 ? OFF_B1 : OFF_B2) + 32 * t + 8 * (r >> 2) + 4 * hh + (r & 3)];
    }
    if (lane < 8) {
        C->shift[lane] = lane < NF ? P[OFF_SHIFT + lane] : 0.f;
        C->scale[lane] = lane < NF ? P[OFF_SCALE + lane] : 0.f;
    }
    if (lane == 0) {
        C->b3 = P[OFF_B3];
        C->out_scale = P[OFF_OUT];
        C->pad[0] = C->pad[1] = 0.f;
    }
}

// Raw features 4h..4h+3 of sample base + p (0 past the sample or feature count).
__device__ __forceinline__ void load_features(const float* __restrict__ feat, int64_t n, int64_t base, float fr[4]) {
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const int64_t s = base + p;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = 4 * h + c;
        fr[c] = (k < NF && s < n) ? feat[s * NF + k] : 0.f;
    }
}

// y of the 32 samples base..base+31 (valid in lanes 0..31 for sample lane)
// from the raw features fr of load_features
// w2(t, c), w3(u, off): the layer-2 A operand of tile t, chunk c, and the
// layer-3 chunk u (off: the tile's opaque zero, for operands read from LDS)
template <typename W2, typename W3>
__device__ __forceinline__ float forward_infer_ops(const InferConst& W, const bf16x4 (&w1)[2], W2 w2, W3 w3,
                                                   const float fr[4], int64_t n, int64_t base) {
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const int64_t s = base + p;
    uint16_t xv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = 4 * h + c;
        float v = 0.f;
        if (k < NF && s < n) {
#pragma clang fp contract(off)
            v = (fr[c] - W.shift[k]) * W.scale[k];
        }
        xv[c] = to_bf16(v);
    }
    const bf16x4 xb = pack4(xv);
    // the bias rows (and operands read from LDS) are re-read every tile: an
    // opaque offset keeps the compiler from holding them in registers across
    // the tile loop (64 for the biases)
    int boff = 0;
    asm volatile("" : "+v"(boff));
    const float* bp = &W.bperm[0][0][h][0] + boff;
    f32x16 z1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) z1[t] = mfma(w1[t], xb, *reinterpret_cast<const f32x16*>(bp + 32 * t));
    bf16x8 hb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) hb[c] = relu_bf16x8(z1[c >> 1], 8 * (c & 1));
    // layer 2 one 32-row tile at a time, each followed by its two layer-3
    // chunks (row 0 of the product holds h2 . w3 for the tile's 32 samples,
    // register 0 of lanes 0..31)
    f32x16 d = {};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16 acc = *reinterpret_cast<const f32x16*>(bp + 64 + 32 * t);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2(t, c, boff), hb[c], acc, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 2; ++u)
            d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w3(2 * t + u, boff), relu_bf16x8(acc, 8 * u), d, 0, 0, 0);
    }
    return (d[0] + W.b3) * W.out_scale;
}

// every operand in registers (the forward pass: 124 VGPRs, four waves per SIMD)
__device__ __forceinline__ float forward_infer(const InferConst& W, const InferRegs& R, const float fr[4], int64_t n,
                                               int64_t base) {
    return forward_infer_ops(
        W, R.w1, [&](int t, int c, int) { return R.w2[t][c]; }, [&](int u, int) { return R.w3[u]; }, fr, n, base);
}

// The layer-2 and layer-3 operands of every lane in LDS, chunk k of lane l
// at [k][l] (w2[t][c] at k = 4 t + c, w3[u] at k = 8 + u): 16-byte reads
// that 64 lanes make at 64 consecutive addresses.  Read per tile (through
// the tile's opaque zero, so that the compiler does not keep them in
// registers across the loop), they take 36 VGPRs off the warm-start pass,
// which then holds four waves per SIMD instead of three.
constexpr int kLdsChunks = 12;
static_assert(sizeof(bf16x8) == 16 && offsetof(InferRegs, w2) == 16 && offsetof(InferRegs, w3) == 144,
              "operand image layout");

// stage the chunks of the image (dwords 4.. of every lane) into img; w1 stays in registers
__device__ __forceinline__ void stage_operands(const uint32_t* __restrict__ packed, bf16x8 (*img)[64], bf16x4 (&w1)[2]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* w = reinterpret_cast<uint32_t*>(&w1[0]);
#pragma unroll
    for (int d = 0; d < 4; ++d) w[d] = packed[d * 64 + lane];
    for (int k = wave; k < kLdsChunks; k += (int)(blockDim.x >> 6)) {
        u32x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = packed[(4 + 4 * k + e) * 64 + lane];
        img[k][lane] = __builtin_bit_cast(bf16x8, v);
    }
}

__device__ __forceinline__ float forward_infer_lds(const InferConst& W, const bf16x8 (*img)[64], const bf16x4 (&w1)[2],
                                                   const float fr[4], int64_t n, int64_t base) {
    const int lane = threadIdx.x & 63;
    return forward_infer_ops(
        W, w1, [&](int t, int c, int off) { return img[4 * t + c][lane + off]; },
        [&](int u, int off) { return img[8 + u][lane + off]; }, fr, n, base);
}

__global__ void __launch_bounds__(256) k_mlp_forward(const uint32_t* __restrict__ packed,
                                                     const float* __restrict__ feat, int64_t n,
                                                     float* __restrict__ y) {
    __shared__ InferConst W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < kConstWords; q += blockDim.x)
        reinterpret_cast<uint32_t*>(&W)[q] = packed[64 * kImageWords + q];
    InferRegs R;
    uint32_t* img = reinterpret_cast<uint32_t*>(&R);
#pragma unroll
    for (int d = 0; d < kImageWords; ++d) img[d] = packed[d * 64 + lane];
    __syncthreads();
    const int64_t tiles = (n + 31) / 32, stride = (int64_t)gridDim.x * 4;
    // the next tile's features are loaded while this tile is computed
    float cur[4] = {0.f, 0.f, 0.f, 0.f};
    int64_t t = (int64_t)blockIdx.x * 4 + wave;
    if (t < tiles) load_features(feat, n, 32 * t, cur);
    for (; t < tiles; t += stride) {
        float nxt[4] = {0.f, 0.f, 0.f, 0.f};
        if (t + stride < tiles) load_features(feat, n, 32 * (t + stride), nxt);
        const float out = forward_infer(W, R, cur, n, 32 * t);
        const int64_t s = 32 * t + lane;
        if (lane < 32 && s < n) y[s] = out;
#pragma unroll
        for (int c = 0; c < 4; ++c) cur[c] = nxt[c];
    }
}

// The learned warm start in one pass (when no training trace is recorded):
// each particle's features from its fields, the network, and the start
// stiffness kappa = K0 = max(0, y alpha rho0 / dt^2), K = 0, x.w = K0 / rho,
// as k_features and k_warm_learned compute them except that a division by
// a constant (rho0, alpha_ref, 26, dt^2 / rho0 ...) is a product with its
// FP32 reciprocal here, cf below (within two units in the last place: the
// IEEE divisions were a third of the pass's vector instructions).
// Lane half 0 holds features 0..3 of its sample, half 1 feature 4.
__device__ __forceinline__ void load_fields(int64_t n, int64_t base, const float* __restrict__ rho,
                                            const float* __restrict__ alpha, const float* __restrict__ K,
                                            const uint32_t* __restrict__ ncnt, const uint32_t* __restrict__ bcnt,
                                            const float* __restrict__ d, const Kern& kc, const float cf[5],
                                            float fr[4], float raw[3]) {
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const int64_t i = base + p;
    fr[0] = fr[1] = fr[2] = fr[3] = 0.f;
    raw[0] = raw[1] = raw[2] = 0.f;
    if (i >= n) return;
    const float a = alpha[i];
    if (h == 0) {   // these lanes also store the start: rho, alpha and K stay in registers for it
        const float r = rho[i], k = K[i];
        fr[0] = (r - kc.rho0) * cf[0];
        fr[1] = d[i] * cf[1];
        fr[2] = (float)(ncnt[i] + bcnt[i]) * (1.0f / 26.0f);
        fr[3] = a > 0.0f ? k * cf[2] / a : 0.0f;
        raw[0] = r;
        raw[1] = a;
        raw[2] = k;
    } else {
        fr[0] = a * cf[3];
    }
}

__global__ void __launch_bounds__(256) k_mlp_warm_start(const uint32_t* __restrict__ packed, int64_t n,
                                                        float4* __restrict__ x, const float* __restrict__ rho,
                                                        const float* __restrict__ alpha, float* __restrict__ K,
                                                        float* __restrict__ kappa, const uint32_t* __restrict__ ncnt,
                                                        const uint32_t* __restrict__ bcnt, const float* __restrict__ d,
                                                        Kern kc, float dt, float alpha_ref, float* __restrict__ Ksave) {
    __shared__ InferConst W;
    __shared__ bf16x8 img[kLdsChunks][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = threadIdx.x; q < kConstWords; q += blockDim.x)
        reinterpret_cast<uint32_t*>(&W)[q] = packed[64 * kImageWords + q];
    bf16x4 w1[2];
    stage_operands(packed, img, w1);
    __syncthreads();
    // 1/rho0, dt/rho0, dt^2/rho0, 1/alpha_ref, rho0/dt^2
    const float cf[5] = {1.0f / kc.rho0, dt / kc.rho0, dt * dt / kc.rho0, 1.0f / alpha_ref, kc.rho0 / (dt * dt)};
    const int64_t tiles = (n + 31) / 32, stride = (int64_t)gridDim.x * 4;
    float cur[4] = {0.f, 0.f, 0.f, 0.f}, craw[3] = {0.f, 0.f, 0.f};
    int64_t t = (int64_t)blockIdx.x * 4 + wave;
    if (t < tiles) load_fields(n, 32 * t, rho, alpha, K, ncnt, bcnt, d, kc, cf, cur, craw);
    for (; t < tiles; t += stride) {
        float nxt[4] = {0.f, 0.f, 0.f, 0.f}, nraw[3] = {0.f, 0.f, 0.f};
        if (t + stride < tiles)
            load_fields(n, 32 * (t + stride), rho, alpha, K, ncnt, bcnt, d, kc, cf, nxt, nraw);
        const float yv = forward_infer_lds(W, img, w1, cur, n, 32 * t);
        const int64_t i = 32 * t + lane;
        if (lane < 32 && i < n) {   // rho, alpha, K of particle i from the feature loads
            const float k0 = fmaxf(yv * craw[1] * cf[4], 0.0f);
            kappa[i] = k0;
            if (Ksave) Ksave[i] = craw[2];
            K[i] = 0.0f;
            x[i].w = k0 / craw[0];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) cur[c] = nxt[c];
#pragma unroll
        for (int c = 0; c < 3; ++c) craw[c] = nraw[c];
    }
}

// ---------------------------------------------------------------- training
// One wave per workgroup.  Partial gradient (packed like the parameters) and
// FP64 loss sum of this workgroup's tiles go to part[blockIdx.x].
__global__ void __launch_bounds__(64) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ feat,
                                                 const float* __restrict__ target, int64_t n,
                                                 float* __restrict__ part, double* __restrict__ loss_part) {
    __shared__ WeightsLDS W;
    __shared__ alignas(16) uint16_t dz2t[H][32];
    __shared__ alignas(16) uint16_t dz1t[H][32];
    __shared__ alignas(16) uint16_t h1t[H][32];
    __shared__ float h2t[H][32], xf[8][32], dzs[32];
    load_weights(W, P, true);
    AOps A;
    load_aops(W, A);
    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const float inv_out = 1.0f / W.out_scale;
    f32x16 gW2[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) gW2[a][b][r] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, gW1[NF] = {0.f, 0.f, 0.f, 0.f, 0.f};
    double loss = 0.0;
    const int64_t tiles = (n + 31) / 32;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = 32 * tile, s = base + p;
        Fwd f;
        forward_tile(W, A, feat, n, base, f);
        // dz = 2 (z - t/out_scale) / n for real samples
        float dz = 0.f;
        if (s < n) {
            const float r = f.z - target[s] * inv_out;
            dz = 2.0f * r / (float)n;
            if (h == 0) loss += (double)r * (double)r;
        }
        if (h == 0) dzs[p] = dz;
        // stash x (FP32 of the bf16 value) and h1^T, h2^T for the row sums and the GEMM
#pragma unroll
        for (int c = 0; c < 4; ++c) xf[4 * h + c][p] = from_bf16((uint16_t)f.xb[c]);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = 32 * t + drow(r, h);
                h1t[j][p] = (uint16_t)f.h1[t][r >> 2][r & 3];
                h2t[j][p] = f.h2[t][r];
            }
        // dZ2^T = bf16(dz w3 [z2 > 0]) in registers (B operands of W2^T) and in LDS
        bf16x4 dz2[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                uint16_t q[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = 4 * cc + u, j = 32 * t + drow(r, h);
                    q[u] = to_bf16(f.z2[t][r] > 0.f ? dz * W.w3[j] : 0.f);
                    dz2t[j][p] = q[u];
                }
                dz2[t][cc] = pack4(q);
            }
        // dH1^T = W2^T dZ2^T, dZ1^T = bf16(dH1^T [z1 > 0])
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16 c;
#pragma unroll
            for (int r = 0; r < 16; ++r) c[r] = 0.f;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bf16x4 a = load4(&W.W2t[(32 * t + p) * H + 8 * b + 4 * h]);
                c = mfma(a, dz2[b >> 2][b & 3], c);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = 32 * t + drow(r, h);
                dz1t[j][p] = to_bf16(f.z1[t][r] > 0.f ? c[r] : 0.f);
            }
        }
        __syncthreads();
        // gW2[j2][j1] += sum_p dZ2^T[j2][p] H1^T[j1][p]: K = the tile's 32 samples
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            bf16x4 Ag[2], Bg[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                Ag[t] = load4(&dz2t[32 * t + p][8 * b + 4 * h]);
                Bg[t] = load4(&h1t[32 * t + p][8 * b + 4 * h]);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) gW2[t][u] = mfma(Ag[t], Bg[u], gW2[t][u]);
        }
        // row sums: thread j owns hidden unit j
        {
            const int j = lane;
            float s1 = 0.f, s2 = 0.f, s3 = 0.f, sw[NF] = {0.f, 0.f, 0.f, 0.f, 0.f};
            for (int q = 0; q < 32; ++q) {
                const float d1 = from_bf16(dz1t[j][q]);
                s1 += d1;
                s2 += from_bf16(dz2t[j][q]);
                s3 += h2t[j][q] * dzs[q];
#pragma unroll
                for (int k = 0; k < NF; ++k) sw[k] += d1 * xf[k][q];
            }
            gb1 += s1;
            gb2 += s2;
            gw3 += s3;
#pragma unroll
            for (int k = 0; k < NF; ++k) gW1[k] += sw[k];
            if (j == 0) {
                float sd = 0.f;
                for (int q = 0; q < 32; ++q) sd += dzs[q];
                gb3 += sd;
            }
        }
        __syncthreads();
    }
    // write this workgroup's partial gradient
    float* o = part + (size_t)blockIdx.x * NPARAM;
    const int j = lane;
#pragma unroll
    for (int k = 0; k < NF; ++k) o[OFF_W1 + j * NF + k] = gW1[k];
    o[OFF_B1 + j] = gb1;
    o[OFF_B2 + j] = gb2;
    o[OFF_W3 + j] = gw3;
    if (j == 0) o[OFF_B3] = gb3;
    if (j < 2 * NF + 1) o[OFF_SHIFT + j] = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) o[OFF_W2 + (32 * t + drow(r, h)) * H + 32 * u + p] = gW2[t][u][r];
    // FP64 loss of the wave (lanes 0..31 hold one sample each)
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
    if (lane == 0) loss_part[blockIdx.x] = loss;
}

__global__ void k_mlp_grad_finish(const float* __restrict__ part, int nblk, float* __restrict__ grad,
                                  const double* __restrict__ loss_part, double* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPARAM) {
        float g = 0.f;
        for (int b = 0; b < nblk; ++b) g += part[(size_t)b * NPARAM + i];
        grad[i] = g;
    }
    if (i == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += loss_part[b];
        *loss = s;
    }
}

// Adam (Kingma and Ba) on the trainable entries; bias-correction denominators
// c1 = 1 - beta1^t, c2 = 1 - beta2^t come from the host.
__global__ void k_mlp_adam(float* __restrict__ P, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= OFF_SHIFT) return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * g;
    const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

constexpr int kMlpGradBlocks = 256;
constexpr int NPARAM_PUBLIC = NPARAM;

int mlp_param_count() { return NPARAM; }
int mlp_grad_blocks() { return kMlpGradBlocks; }

int mlp_packed_words() { return kPackedWords; }

hipError_t launch_mlp_pack(const float* P, uint32_t* packed, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, s, P, packed);
    return hipGetLastError();
}

namespace {
// Workgroups of 256 threads of `kernel` that the current device holds at
// once (its compute units times the occupancy the kernel's registers
// allow), looked up once per device; 0 when the runtime cannot say.  A
// grid-stride pass launched with exactly that many runs in one wave of
// workgroups: one more would leave a partial second round at the end.
constexpr int kMaxResidentDevices = 64;
int64_t resident_blocks(const void* kernel, std::atomic<int64_t>* cache) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxResidentDevices) return 0;
    int64_t v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || ncu <= 0 || per <= 0)
        return 0;
    v = (int64_t)ncu * per;
    cache[dev].store(v, std::memory_order_relaxed);
    return v;
}
std::atomic<int64_t> g_resident_warm[kMaxResidentDevices], g_resident_forward[kMaxResidentDevices];

// at most one resident round of four-wave workgroups (1024 if the runtime cannot say)
int64_t mlp_grid(int64_t n, const void* kernel, std::atomic<int64_t>* cache) {
    const int64_t tiles = (n + 31) / 32;
    int64_t cap = resident_blocks(kernel, cache);
    if (cap <= 0) cap = 1024;
    return std::min((tiles + 3) / 4, cap);
}
}  // namespace

hipError_t launch_mlp_warm_start(const uint32_t* packed, int64_t n, float4* x, const float* rho, const float* alpha,
                                 float* K, float* kappa, const uint32_t* ncnt, const uint32_t* bcnt, const float* d,
                                 Kern kc, float dt, float alpha_ref, float* Ksave, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = mlp_grid(n, reinterpret_cast<const void*>(k_mlp_warm_start), g_resident_warm);
    hipLaunchKernelGGL(k_mlp_warm_start, dim3((uint32_t)blocks), dim3(256), 0, s, packed, n, x, rho, alpha, K, kappa,
                       ncnt, bcnt, d, kc, dt, alpha_ref, Ksave);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint32_t* packed, const float* feat, int64_t n, float* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // weights staged once per workgroup, so as few workgroups as fill the device
    const int64_t blocks = mlp_grid(n, reinterpret_cast<const void*>(k_mlp_forward), g_resident_forward);
    hipLaunchKernelGGL(k_mlp_forward, dim3((uint32_t)blocks), dim3(256), 0, s, packed, feat, n, y);
    return hipGetLastError();
}

// grad[NPARAM] and *loss_sum (sum of squared residuals in units of out_scale)
hipError_t launch_mlp_grad(const float* P, const float* feat, const float* target, int64_t n, float* part,
                           double* loss_part, float* grad, double* loss_sum, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(kMlpGradBlocks), dim3(64), 0, s, P, feat, target, n, part, loss_part);
    hipLaunchKernelGGL(k_mlp_grad_finish, dim3((NPARAM + 255) / 256), dim3(256), 0, s, part, kMlpGradBlocks, grad,
                       loss_part, loss_sum);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, grad, m, v, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace sph

// ---------------------------------------------------------------------------
// Allocation-free MLP gradient.  The per-workgroup partial gradients and FP64
// loss partials live in a file-scope device array instead of buffers that
// sph_mlp_create allocates.  Every launch writes all kMlpGradBlocks partial
// slots before the finishing kernel reads them, so nothing in it has to start
// at zero.  Each device holds its own copy of the array; host code reaches it
// only through the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
#include <mutex>

#include "sph.h"

namespace {
constexpr size_t kNoAllocPartBytes = sizeof(float) * (size_t)sph::kMlpGradBlocks * sph::NPARAM_PUBLIC;
constexpr size_t kNoAllocBytes = kNoAllocPartBytes + sizeof(double) * sph::kMlpGradBlocks;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];   // device address of `scratch` on each device (null until first use)
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// The address of `scratch` on the current device, looked up once per device.
static int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPH_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPH_ERR_DEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SPH_OK;
}

extern "C" int sph_mlp_grad_noalloc(const float* params, const float* features, const float* targets, int64_t n,
                                    float* grad, double* loss_sum, void* hip_stream) {
    if (!params || !features || !targets || !grad || !loss_sum || n <= 0) return SPH_ERR_INVALID;
    if (n > SPH_MLP_NOALLOC_MAX_ROWS) return SPH_ERR_INVALID;
    void* base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != SPH_OK) return rc;
    float* part = static_cast<float*>(base);
    double* loss_part = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kNoAllocPartBytes);
    return sph::launch_mlp_grad(params, features, targets, n, part, loss_part, grad, loss_sum,
                                (hipStream_t)hip_stream) == hipSuccess
               ? SPH_OK
               : SPH_ERR_DEVICE;
}
