// Device-side pieces of the learned EOS seed network shared by the network
// kernels and the hydro stage kernel (see tdh_mlp.hip for the layouts).
#pragma once
#include "tdh_internal.hpp"

namespace tdh {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 128, OFF_W2 = 192, OFF_B2 = 192 + 4096, OFF_W3 = OFF_B2 + 64, OFF_B3 = OFF_W3 + 64;
constexpr int NPARAM = OFF_B3 + 1;


__device__ __forceinline__ short to_bf16(float f) {
  return __builtin_bit_cast(short, (__bf16)f);  // round to nearest even (v_cvt_pk_bf16_f32)
}
__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }
__device__ __forceinline__ float round_bf16(float f) { return from_bf16(to_bf16(f)); }

// layer 1 for the 64 samples of this wave, directly in the A-operand layout
// of the hidden-layer product: a[mt][kt] holds h1[q = 16 mt + l%16][k = 32 kt + 8 (l/16) + e]
__device__ __forceinline__ void layer1_A(const MlpDev &w, float xb0, float xb1, bf16x8 (&a)[4][2]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int q = 16 * mt + (l & 15);
    const float x0 = __shfl(xb0, q, 64), x1 = __shfl(xb1, q, 64);
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kt + 8 * (l >> 4) + e;
        float z = w.b1[k];
        z += from_bf16(w.w1b[2 * k]) * x0;
        z += from_bf16(w.w1b[2 * k + 1]) * x1;
        a[mt][kt][e] = to_bf16(fmaxf(z, 0.0f));
      }
    }
  }
}

// hidden-layer pre-activations Z2[q][o] in D layout: acc[mt][nt][r] at
// q = 16 mt + 4 (l/16) + r, o = 16 nt + l%16
__device__ __forceinline__ void layer2(const MlpDev &w, const bf16x8 (&a)[4][2], f32x4 (&acc)[4][4]) {
  const int l = threadIdx.x & 63;
  bf16x8 bop[4][2];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      bop[nt][kt] = *(const bf16x8 *)(w.w2b + (16 * nt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][0], bop[nt][0], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][1], bop[nt][1], c, 0, 0, 0);
      acc[mt][nt] = c;
    }
}

// y for this lane's own sample (q = lane), from the D-layout pre-activations
__device__ __forceinline__ float layer3(const MlpDev &w, const f32x4 (&acc)[4][4]) {
  const int l = threadIdx.x & 63;
  float part[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int o = 16 * nt + (l & 15);
        const float h = round_bf16(fmaxf(acc[mt][nt][r] + w.b2[o], 0.0f));
        s += from_bf16(w.w3b[o]) * h;
      }
      // sum over the 16 lanes of this row group (the 16 output columns)
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      part[mt][r] = s;
    }
  // sample q = l lives in row group (l%16)/4, tile mt = l/16, row r = l%4
  float y = 0.0f;
  const int src = 16 * ((l & 15) >> 2);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = __shfl(part[mt][r], src, 64);
      if (mt == (l >> 4) && r == (l & 3)) y = v;
    }
  return y + w.b3[0];
}

// whole forward pass for the wave; every lane of the wave must call it
__device__ __forceinline__ float mlp_wave_forward(const MlpDev &w, float x0, float x1) {
  bf16x8 a[4][2];
  f32x4 acc[4][4];
  layer1_A(w, round_bf16(x0), round_bf16(x1), a);
  layer2(w, a, acc);
  return layer3(w, acc);
}

// Inference forward pass with all three layers on the matrix cores.  Each lane
// passes its own sample's normalised inputs and gets its output.  The hidden
// activations are kept transposed (unit x sample), and the units are numbered
// so that each product's output tile is, lane by lane, the operand the next
// product needs:
//   layer 1, tile (mt, nt): A = W1 rows 16 mt.. in slots e = 0, 1 of every
//     lane group, B = the own (x0, x1) of lane group nt's lanes in those slots
//     (zero in the other groups), accumulator = b1; D holds
//     z1[h = 16 mt + 4 (l/16) + r][q = 16 nt + l%16];
//   layer 2, tile (mo, nt): B for K tile kt is this lane's D of layer-1 tiles
//     mt = 2 kt, 2 kt + 1 (after ReLU and bf16), i.e. contraction slot
//     kappa = 32 kt + 8 (l/16) + e holds hidden unit
//     h = 16 (2 kt + e/4) + 4 (l/16) + e%4; A = W2 with its columns in that
//     order; accumulator = b2; D holds z2[o = 16 mo + 4 (l/16) + r][q = 16 nt + l%16];
//   layer 3, tile nt: B is built from the layer-2 tiles as layer 2's B from
//     layer 1's; every row of A holds w3 in that contraction order and the
//     accumulator is b3, so every row of D holds the outputs of samples
//     16 nt .. 16 nt + 15, and lane l takes its own from tile nt = l/16.
// The products of bf16 operands are exact in fp32; the sums, biases included,
// are fp32 in the matrix cores' order (mlp_wave_forward adds the bias after
// the products).  Every lane of the wave must call it.
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;

// ReLU and bf16 of a D-layout tile into half `hi` of a B operand.  Rounding to
// nearest keeps the sign, so the ReLU is taken after it, on pairs of bf16 bit
// patterns as 16-bit integers (negative values, -0 included, have the sign
// bit set and become +0; the rest are unchanged): relu(bf16(z)) = bf16(relu(z)).
__device__ __forceinline__ void relu_to_operand(const f32x4 &z, bf16x8 &b, int hi) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const s16x2 zero = {0, 0};
  const s16x2 p = __builtin_elementwise_max(
      __builtin_bit_cast(s16x2, __builtin_convertvector(f32x2{z[0], z[1]}, b16x2)), zero);
  const s16x2 q = __builtin_elementwise_max(
      __builtin_bit_cast(s16x2, __builtin_convertvector(f32x2{z[2], z[3]}, b16x2)), zero);
  b[4 * hi + 0] = p.x;
  b[4 * hi + 1] = p.y;
  b[4 * hi + 2] = q.x;
  b[4 * hi + 3] = q.y;
}

// 8 values of a 64-vector in the contraction order above (K tile kt, lane group g)
__device__ __forceinline__ bf16x8 permuted_row(const short *v, int kt, int g) {
  const bf16x4 lo = *(const bf16x4 *)(v + 32 * kt + 4 * g), hi = *(const bf16x4 *)(v + 32 * kt + 16 + 4 * g);
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

__device__ __forceinline__ f32x4 bias_tile(const float *b, int t, int g) {
  const float4 v = *(const float4 *)(b + 16 * t + 4 * g);
  return f32x4{v.x, v.y, v.z, v.w};
}

// layer-1 operands: A = the two input weights of hidden unit 16 mt + l%16 in
// slots e = 0, 1 of every lane group; B for sample group nt = this lane's own
// (x0, x1) in those slots in lane group nt and zero in the others, so the
// contraction over the four groups picks the samples 16 nt .. 16 nt + 15
__device__ __forceinline__ bf16x8 layer1_weights(const MlpDev &w, int mt, int c) {
  const uint32_t v = *(const uint32_t *)(w.w1b + 2 * (16 * mt + c));
  return __builtin_bit_cast(bf16x8, uint4{v, 0u, 0u, 0u});
}
__device__ __forceinline__ bf16x8 layer1_inputs(uint32_t xpair, int nt, int g) {
  return __builtin_bit_cast(bf16x8, uint4{g == nt ? xpair : 0u, 0u, 0u, 0u});
}
__device__ __forceinline__ uint32_t input_pair(float x0, float x1) {
  return (uint32_t)(uint16_t)to_bf16(x0) | ((uint32_t)(uint16_t)to_bf16(x1) << 16);
}

// l: the lane index (an opaque per-item value inside a larger kernel keeps the
// weight loads next to their use).  One sample group at a time: few registers.
__device__ __forceinline__ float mlp_wave_forward_fast(const MlpDev &w, float x0, float x1, int l) {
  const int g = l >> 4, c = l & 15;
  const uint32_t xp = input_pair(x0, x1);
  const float b3 = w.b3[0];
  float y = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    bf16x8 b2op[2], b3op[2];
    const bf16x8 bx = layer1_inputs(xp, nt, g);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(layer1_weights(w, mt, c), bx, bias_tile(w.b1, mt, g), 0,
                                                              0, 0);
      relu_to_operand(z, b2op[mt >> 1], mt & 1);
    }
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      f32x4 z = bias_tile(w.b2, mo, g);
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
        z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(permuted_row(w.w2b + (16 * mo + c) * H, kt, g), b2op[kt], z,
                                                    0, 0, 0);
      relu_to_operand(z, b3op[mo >> 1], mo & 1);
    }
    f32x4 z3 = {b3, b3, b3, b3};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(permuted_row(w.w3b, kt, g), b3op[kt], z3, 0, 0, 0);
    if (g == nt) y = z3[0];  // this lane's own sample is 16 nt + l%16 = l
  }
  return y;
}

// The same products and sums as mlp_wave_forward_fast (bit for bit), in an
// order that loads every weight once per call: layer 1 for all four sample
// groups first, then each output tile's layer-2 weights serve the four groups.
// Needs more registers; for kernels that have them.
__device__ __forceinline__ float mlp_wave_forward_hoisted(const MlpDev &w, float x0, float x1, int l) {
  const int g = l >> 4, c = l & 15;
  const uint32_t xp = input_pair(x0, x1);
  bf16x8 b2op[4][2], b3op[4][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f32x4 b1 = bias_tile(w.b1, mt, g);
    const bf16x8 a1 = layer1_weights(w, mt, c);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, layer1_inputs(xp, nt, g), b1, 0, 0, 0);
      relu_to_operand(z, b2op[nt][mt >> 1], mt & 1);
    }
  }
#pragma unroll
  for (int mo = 0; mo < 4; ++mo) {
    const bf16x8 a2[2] = {permuted_row(w.w2b + (16 * mo + c) * H, 0, g), permuted_row(w.w2b + (16 * mo + c) * H, 1, g)};
    const f32x4 b2 = bias_tile(w.b2, mo, g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[0], b2op[nt][0], b2, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[1], b2op[nt][1], z, 0, 0, 0);
      relu_to_operand(z, b3op[nt][mo >> 1], mo & 1);
    }
  }
  const bf16x8 a3[2] = {permuted_row(w.w3b, 0, g), permuted_row(w.w3b, 1, g)};
  const float b3 = w.b3[0];
  float y = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 z3 = {b3, b3, b3, b3};
    z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[0], b3op[nt][0], z3, 0, 0, 0);
    z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[1], b3op[nt][1], z3, 0, 0, 0);
    if (g == nt) y = z3[0];
  }
  return y;
}

__device__ __forceinline__ float norm01(double v, double lo, double hi) {
  return (float)(2.0 * (v - lo) / (hi - lo) - 1.0);
}

}  // namespace tdh
