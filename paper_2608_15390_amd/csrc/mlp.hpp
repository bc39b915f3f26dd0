// mlp.hpp -- the per-edge proposal network on matrix cores.
//
// Network: 8 edge features -> 64 (ReLU) -> 64 (ReLU) -> 1 logit.
// Parameters (float, packed): W1[8][64], b1[64], W2[64][64], b2[64],
// w3[64], b3.  Layers 1 and 2 run as bf16 MFMA 16x16x16 tiles over 16
// records at a time with float accumulation; layer 3 is a 64-term dot
// product reduced across lanes.
//
// MFMA 16x16x16 bf16 operand layout (one wave): for lane l, A[i][k] with
// i = l % 16, k = 4 (l / 16) + j; B[k][c] with c = l % 16,
// k = 4 (l / 16) + j; the result D[i][c] with c = l % 16, i = 4 (l / 16) + j
// (j = 0..3).
#pragma once
#include "device.hpp"

namespace pe {

constexpr int kIn = 8, kH = 64;
constexpr int kEtabN = 2048;  // entries of the integer softmax table (larger gaps weigh 0)
// rint(2^24 exp(-d/16)) is 0 from d = 278 on, so the kernels keep only the
// first kEtabLds entries of the table and read 0 beyond them
constexpr int kEtabLds = 288;
constexpr int kNParam = kIn * kH + kH + kH * kH + kH + kH + 1;  // 4801
// offsets into the packed parameter vector
constexpr int kOffW1 = 0, kOffB1 = kIn * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's K = 32 tile: lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
    typedef short s8 __attribute__((ext_vector_type(8)));
    const s8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Weights in matrix-core form, staged once per block in LDS, each lane's
// four B-operand values contiguous (one 8-byte LDS read per MFMA):
//   w1[nt][lane < 32][4] = W1[4 (lane / 16) + j][16 nt + lane % 16] (the K = 16
//     tile's rows 8..15 are zero and not stored),
//   w2[ks][nt][lane][4] = W2[16 ks + 4 (lane / 16) + j][16 nt + lane % 16],
// and float b1, b2, w3, b3.
struct MlpLds {
    short w1[kIn * kH];
    short w2[kH * kH];
    float b1[kH], b2[kH], w3[kH];
    float b3;
};

// The sampling side's LDS block: the network plus the non-zero part of the
// integer softmax table E[d] (values <= 2^24, so 32 bits hold them).
struct LearnedLds {
    MlpLds net;
    uint32_t etab[kEtabLds];
};

// position of W2[r][c] in MlpLds::w2
__device__ __forceinline__ int w2_index(int r, int c) {
    const int ks = r >> 4, nt = c >> 4, lane = 16 * ((r & 15) >> 2) + (c & 15);
    return ((ks * 4 + nt) * 64 + lane) * 4 + (r & 3);
}

// GRID (inference on the grid, parameters already snapped to k/64): W1, b1
// and b2 are staged times 64, so that layers 1 and 2 produce 64 z directly
// and the activations are the grid integers k (see mlp_tile_logit_grid).
template <bool GRID = false>
__device__ void stage_weights(MlpLds *s, const float *P) {
    const float g = GRID ? 64.0f : 1.0f;
    for (int i = threadIdx.x; i < kIn * kH; i += blockDim.x) {
        const int j = i & 3, lane = (i >> 2) & 31, nt = i >> 7;
        s->w1[i] = to_bf16(g * P[kOffW1 + (4 * (lane >> 4) + j) * kH + 16 * nt + (lane & 15)]);
    }
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
        const int r = i >> 6, c = i & 63;
        s->w2[w2_index(r, c)] = to_bf16(P[kOffW2 + i]);
    }
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        s->b1[i] = g * P[kOffB1 + i];
        s->b2[i] = g * P[kOffB2 + i];
        s->w3[i] = P[kOffW3 + i];
    }
    if (threadIdx.x == 0) s->b3 = P[kOffB3];
}

// Per-wave scratch for one 16-record tile: a [16][64] bf16 activation tile.
struct TileLds {
    short h[16 * kH];
};

// Forward of one tile of the float network (training).  `xa` is this
// lane's A operand of the feature tile (record l % 16, features
// 4 (l / 16) .. +3; features 8..15 are zero).  Outputs in D layout: z1[nt],
// z2[nt] (pre-activations, column 16 nt + l % 16, rows 4 (l / 16) + j) and
// the logits of rows 4 (l / 16) + j (complete in the last lane of each
// 16-lane group, l % 16 == 15).
// four consecutive bf16 operands (8-byte aligned)
__device__ __forceinline__ bf16x4 load_b4(const short *p) { return *reinterpret_cast<const bf16x4 *>(p); }

__device__ __forceinline__ void mlp_tile_forward(const MlpLds *W, TileLds *T, bf16x4 xa, f32x4 z1[4],
                                                 f32x4 z2[4], float logit[4]) {
    const int l = lane_id();
    const int c0 = l % 16, r0 = 4 * (l / 16);
    auto act = [](float z) -> float { return z > 0.0f ? z : 0.0f; };
    auto act_bf16 = [&](float z) -> short { return to_bf16(act(z)); };
    // layer 1: [16 x 16] x [16 x 64], the bias as the accumulator's start
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        bf16x4 b = {0, 0, 0, 0};
        if (l < 32) b = load_b4(&W->w1[(nt * 32 + l) * 4]);
        const float bias = W->b1[16 * nt + c0];
        f32x4 acc = {bias, bias, bias, bias};
        acc = mfma16(xa, b, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) T->h[(r0 + j) * kH + 16 * nt + c0] = act_bf16(acc[j]);
        z1[nt] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    // layer 2: [16 x 64] x [64 x 64], A read back from LDS in A layout
    bf16x4 a2[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
        a2[ks] = *reinterpret_cast<const bf16x4 *>(&T->h[c0 * kH + 16 * ks + r0]);
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float bias = W->b2[16 * nt + c0];
        f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const bf16x4 b = load_b4(&W->w2[((ks * 4 + nt) * 64 + l) * 4]);
            acc = mfma16(a2[ks], b, acc);
        }
        const float w3 = W->w3[16 * nt + c0];
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] = part[j] + act(acc[j]) * w3;
        z2[nt] = acc;
    }
    // layer 3: sum the 64 columns over the 16 lanes of each row group (a
    // row-shifted DPP scan: the group total lands in its last lane)
    auto fadd = [](uint32_t a, uint32_t b) { return __float_as_uint(__uint_as_float(a) + __uint_as_float(b)); };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t v = __float_as_uint(part[j]);
        v = fadd(v, dpp<kRowShr1>(0u, v));
        v = fadd(v, dpp<kRowShr2>(0u, v));
        v = fadd(v, dpp<kRowShr4>(0u, v));
        v = fadd(v, dpp<kRowShr8>(0u, v));
        logit[j] = __uint_as_float(v) + W->b3;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Inference on the grid (weights staged with GRID), network transposed:
// each layer computes W^T times the transposed activations, so the weights
// are the A operand and the activations the B operand. The B-layout staging
// of W is exactly the A layout of W^T, and the feature tile xb is the same
// operand as xa above (record l % 16, features 4 (l / 16) + j). One tile's
// result in D layout (rows 4 (l / 16) + j, column l % 16) is the B operand
// of the next layer's K-step as it stands, so the activations stay in
// registers. Each lane ends with the logit of record l % 16: the four rows
// hold partial sums over complementary hidden units, added across rows by
// two lane-swap steps.
// The tile carries everything times 64: with W1, b1 and b2 staged times 64,
// layer 1 yields 64 z1 and an activation is the grid integer
// k = med3(rint(64 z1), 0, 255) (exact in bf16); layer 2 on those integers
// with the unscaled W2 yields 64 z2; layer 3 sums k w3 and scales by 1/64
// at the end. Every product and partial sum is a grid value with at most
// 64 terms, exact in binary32, so neither the scaling nor the order of the
// sums changes a logit: it is the exact value of the snapped network.
__device__ __forceinline__ float mlp_tile_logit_grid(const MlpLds *W, bf16x4 xb) {
    const int l = lane_id();
    const int g4 = 4 * (l / 16);
    auto act = [](float z) -> float { return __builtin_amdgcn_fmed3f(rintf(z), 0.0f, 255.0f); };
    bf16x4 h1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        bf16x4 a = {0, 0, 0, 0};
        if (l < 32) a = load_b4(&W->w1[(nt * 32 + l) * 4]);
        f32x4 acc = *reinterpret_cast<const f32x4 *>(&W->b1[16 * nt + g4]);
        acc = mfma16(a, xb, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) h1[nt][j] = (short)(__float_as_uint(act(acc[j])) >> 16);
    }
    // layer 2 on K = 32 tiles. The contraction pairs A and B by slot, so
    // slot (g, j) of block kk may stand for any layer-1 unit as long as both
    // operands agree: slots j < 4 take unit 32 kk + 4 g + j (layer 1's tile
    // 2 kk as this lane holds it), slots j >= 4 unit 32 kk + 16 + 4 g + j - 4
    // (tile 2 kk + 1). Both operands are then concatenations of what the
    // K = 16 layout already has in place. Every product and partial sum is
    // exact on the grid, so the grouping does not change the logit.
    float part = 0.0f;
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = *reinterpret_cast<const f32x4 *>(&W->b2[16 * nt + g4]);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bf16x8 a = cat8(load_b4(&W->w2[((2 * kk * 4 + nt) * 64 + l) * 4]),
                                  load_b4(&W->w2[(((2 * kk + 1) * 4 + nt) * 64 + l) * 4]));
            acc = mfma32(a, cat8(h1[2 * kk], h1[2 * kk + 1]), acc);
        }
        const f32x4 w3 = *reinterpret_cast<const f32x4 *>(&W->w3[16 * nt + g4]);
#pragma unroll
        for (int j = 0; j < 4; ++j) part = __builtin_fmaf(act(acc[j]), w3[j], part);
    }
    // rows 0+1 and 2+3, then the two halves
    const uint32_t pu = __float_as_uint(part);
    const auto s16 = __builtin_amdgcn_permlane16_swap(pu, pu, false, false);
    part = __uint_as_float(s16[0]) + __uint_as_float(s16[1]);
    const uint32_t qu = __float_as_uint(part);
    const auto s32 = __builtin_amdgcn_permlane32_swap(qu, qu, false, false);
    part = __uint_as_float(s32[0]) + __uint_as_float(s32[1]);
    return part * (1.0f / 64.0f) + W->b3;
}

// ------------------------------------------------------------- training
// Feature tile A operand for records [r, r + 16) of X[n][8] (zero past n)
__device__ __forceinline__ bf16x4 load_x_tile(const float *X, int64_t n, int64_t r) {
    const int l = lane_id();
    const int64_t row = r + l % 16;
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = 4 * (l / 16) + j;
        a[j] = (row < n && k < kIn) ? to_bf16(X[row * kIn + k]) : (short)0;
    }
    return a;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float *P, const float *X, int64_t n, float *logits) {
    __shared__ MlpLds W;
    __shared__ TileLds tiles[4];
    stage_weights(&W, P);
    __syncthreads();
    const int wave = threadIdx.x / kWave, l = lane_id();
    const int64_t tiles_total = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tiles_total; t += (int64_t)gridDim.x * 4) {
        f32x4 z1[4], z2[4];
        float lg[4];
        mlp_tile_forward(&W, &tiles[wave], load_x_tile(X, n, 16 * t), z1, z2, lg);
        if (l % 16 == 15)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = 16 * t + 4 * (l / 16) + j;
                if (row < n) logits[row] = lg[j];
            }
    }
}

// Per group g in [g0, g1): softmax of its logits, d loss / d logit =
// (softmax - target) / G and the group's cross-entropy added to *loss.
// Records are indexed relative to r0 = gstart[g0] (the window's first).
__global__ void k_softmax_xent(const float *logits, const float *targets, const int64_t *gstart,
                               const int32_t *ginfo, int64_t g0, int64_t g1, float *dlogits, double *loss) {
    const int64_t g = g0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lg = 0.0;
    if (g < g1) {
        const int64_t s = gstart[g] - gstart[g0];
        const int32_t k = ginfo[4 * g];
        const float inv_g = 1.0f / (float)(g1 - g0);
        float mx = -3.0e38f;
        for (int32_t i = 0; i < k; ++i) mx = fmaxf(mx, logits[s + i]);
        float sum = 0.0f;
        for (int32_t i = 0; i < k; ++i) sum += expf(logits[s + i] - mx);
        for (int32_t i = 0; i < k; ++i) {
            const float p = expf(logits[s + i] - mx) / sum;
            const float y = targets[gstart[g0] + s + i];
            dlogits[s + i] = (p - y) * inv_g;
            if (y > 0.0f) lg -= (double)y * ((double)(logits[s + i] - mx) - log((double)sum));
        }
        lg /= (double)(g1 - g0);
    }
    // one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lg += __shfl_xor(lg, o);
    if (lane_id() == 0) atomicAdd(loss, lg);
}

// Backward over the n records of X (dlogits indexed alike): gradients of
// all parameters, accumulated per wave in registers and stored as that
// wave's partial, parts[global wave][kNParam] (summed in a fixed order by
// the caller, so gradients are reproducible).
__global__ void __launch_bounds__(256) k_mlp_backward(const float *P, const float *X, const float *dlogits,
                                                      int64_t n, float *parts) {
    __shared__ MlpLds W;
    __shared__ TileLds tiles[4];
    stage_weights(&W, P);
    __syncthreads();
    const int wave = threadIdx.x / kWave, l = lane_id();
    const int c0 = l % 16, q0 = 4 * (l / 16);
    TileLds *T = &tiles[wave];
    f32x4 gW2[4][4], gW1[4];
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0, 0, 0, 0};
    }
    const int64_t tiles_total = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tiles_total; t += (int64_t)gridDim.x * 4) {
        const int64_t base = 16 * t;
        f32x4 z1[4], z2[4];
        float lg[4];
        mlp_tile_forward(&W, T, load_x_tile(X, n, base), z1, z2, lg);
        float dl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = base + q0 + j;
            dl[j] = row < n ? dlogits[row] : 0.0f;
            if (c0 == 0) gb3 += dl[j];
        }
        // dZ2 = dl w3 1[z2 > 0]; gradients of w3, b2; dW2 = H1^T dZ2
        f32x4 dz2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const float w3c = W.w3[16 * nt + c0];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float h2 = z2[nt][j] > 0.0f ? z2[nt][j] : 0.0f;
                gw3[nt] += h2 * dl[j];
                dz2[nt][j] = z2[nt][j] > 0.0f ? dl[j] * w3c : 0.0f;
                gb2[nt] += dz2[nt][j];
            }
        }
        bf16x4 h1a[4], dz2b[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h1a[nt][j] = T->h[(q0 + j) * kH + 16 * nt + c0];  // H1 in D layout = A of H1^T
                dz2b[nt][j] = to_bf16(dz2[nt][j]);
            }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gW2[mt][nt] = mfma16(h1a[mt], dz2b[nt], gW2[mt][nt]);
        // dH1 = dZ2 W2^T: dZ2 to A layout through LDS
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) T->h[(q0 + j) * kH + 16 * nt + c0] = dz2b[nt][j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        bf16x4 dza[4];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs) dza[cs] = *reinterpret_cast<const bf16x4 *>(&T->h[c0 * kH + 16 * cs + q0]);
        bf16x4 dz1b[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int cs = 0; cs < 4; ++cs) {
                bf16x4 b;  // B[c][k] = W2[k][c], k = 16 nt + c0, c = 16 cs + q0 + j
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = W.w2[w2_index(16 * nt + c0, 16 * cs + q0 + j)];
                acc = mfma16(dza[cs], b, acc);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float d = z1[nt][j] > 0.0f ? acc[j] : 0.0f;
                gb1[nt] += d;
                dz1b[nt][j] = to_bf16(d);
            }
        }
        // dW1 = X^T dZ1 (A[k][i] = X[base + i][k], rows k >= 8 zero)
        bf16x4 xt;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = base + q0 + j;
            xt[j] = (row < n && c0 < kIn) ? to_bf16(X[row * kIn + c0]) : (short)0;
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gW1[nt] = mfma16(xt, dz1b[nt], gW1[nt]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    // this wave's partial: every parameter written by exactly one lane
    float *grad = parts + ((size_t)blockIdx.x * 4 + wave) * kNParam;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                grad[kOffW2 + (16 * mt + q0 + j) * kH + 16 * nt + c0] = gW2[mt][nt][j];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (q0 + j < kIn) grad[kOffW1 + (q0 + j) * kH + 16 * nt + c0] = gW1[nt][j];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        float a = gb1[nt], b = gb2[nt], c = gw3[nt];
        a += __shfl_xor(a, 16); a += __shfl_xor(a, 32);
        b += __shfl_xor(b, 16); b += __shfl_xor(b, 32);
        c += __shfl_xor(c, 16); c += __shfl_xor(c, 32);
        if (l < 16) {
            grad[kOffB1 + 16 * nt + c0] = a;
            grad[kOffB2 + 16 * nt + c0] = b;
            grad[kOffW3 + 16 * nt + c0] = c;
        }
    }
    float s3 = gb3;
    for (int o = 32; o > 0; o >>= 1) s3 += __shfl_xor(s3, o);
    if (l == 0) grad[kOffB3] = s3;
}

__global__ void k_adam(float *P, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.0f - b1) * gi;
    v[i] = b2 * v[i] + (1.0f - b2) * gi * gi;
    const float mh = m[i] / c1, vh = v[i] / c2;
    P[i] = P[i] - lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_fill_f32n(int64_t n, float *p, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Inference grid of the learned proposal: every parameter snapped to the
// nearest multiple of 1/64 in [-127/64, 127/64]; *bad set for non-finite input.
__global__ void k_quantize_params(const float *src, float *dst, int n, int32_t *bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float p = src[i];
    if (!__builtin_isfinite(p)) { atomicOr(bad, 1); dst[i] = 0.0f; return; }
    float k = rintf(p * 64.0f);
    k = k < -127.0f ? -127.0f : (k > 127.0f ? 127.0f : k);
    dst[i] = k * (1.0f / 64.0f);
}

// integer softmax table E[d] = rint(2^24 exp(-d/16)), d = 0 .. kEtabN-1
__global__ void k_etab(int64_t *E) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < kEtabN) E[d] = (int64_t)rint(16777216.0 * exp(-(double)d / 16.0));
}

}  // namespace pe
