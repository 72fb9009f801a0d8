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

// Inference forward pass with every layer but the output on the matrix cores.
// Each lane passes its own sample's normalised inputs and gets its output.
// The hidden activations are kept transposed, H1^T[k][q] (hidden unit x
// sample), and the hidden units are numbered so that the output tile of the
// first product is, lane by lane, the operand the second product needs:
//   layer 1, tile (mt, nt): A = W1 rows 16 mt.. placed in the K slots of lane
//     group nt (zero elsewhere), B = every lane's own (x0, x1) in its slots
//     e = 0, 1; D holds z1[h = 16 mt + 4 (l/16) + r][q = 16 nt + l%16];
//   layer 2, tile (mo, nt): B for K tile kt is this lane's D of layer-1 tiles
//     mt = 2 kt, 2 kt + 1 (after bias, ReLU, bf16), i.e. contraction slot
//     kappa = 32 kt + 8 (l/16) + e holds hidden unit
//     h = 16 (2 kt + e/4) + 4 (l/16) + e%4; A = W2 with its columns in that order;
//     D holds z2[o = 16 mo + 4 (l/16) + r][q = 16 nt + l%16];
//   layer 3 sums w3[o] h2 over this lane's 16 outputs, then over the four lane
//     groups.
// Same function as mlp_wave_forward (bf16 operands, fp32 sums and biases); the
// fp32 sums are taken in another order.  l: the lane index (an opaque per-item
// value inside a larger kernel keeps the weight loads next to their use).
__device__ __forceinline__ float mlp_wave_forward_fast(const MlpDev &w, float x0, float x1, int l) {
  typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
  const int g = l >> 4, c = l & 15;
  bf16x8 bx = {0, 0, 0, 0, 0, 0, 0, 0};
  bx[0] = to_bf16(x0);
  bx[1] = to_bf16(x1);
  float y = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    // layer 1 for samples 16 nt .. 16 nt + 15, hidden layer in layer-2 B layout
    bf16x8 b2op[2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      bf16x8 a1 = {0, 0, 0, 0, 0, 0, 0, 0};
      if (g == nt) {
        a1[0] = w.w1b[2 * (16 * mt + c)];
        a1[1] = w.w1b[2 * (16 * mt + c) + 1];
      }
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bx, z, 0, 0, 0);
      const float4 b1 = *(const float4 *)(w.b1 + 16 * mt + 4 * g);
      b2op[mt >> 1][4 * (mt & 1) + 0] = to_bf16(fmaxf(z[0] + b1.x, 0.0f));
      b2op[mt >> 1][4 * (mt & 1) + 1] = to_bf16(fmaxf(z[1] + b1.y, 0.0f));
      b2op[mt >> 1][4 * (mt & 1) + 2] = to_bf16(fmaxf(z[2] + b1.z, 0.0f));
      b2op[mt >> 1][4 * (mt & 1) + 3] = to_bf16(fmaxf(z[3] + b1.w, 0.0f));
    }
    // layer 2 and the output layer
    float s = 0.0f;
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        const short *row = w.w2b + (16 * mo + c) * H + 32 * kt + 4 * g;
        const bf16x4 lo = *(const bf16x4 *)row, hi = *(const bf16x4 *)(row + 16);
        const bf16x8 a2 = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2op[kt], z, 0, 0, 0);
      }
      const float4 b2 = *(const float4 *)(w.b2 + 16 * mo + 4 * g);
      const bf16x4 w3 = *(const bf16x4 *)(w.w3b + 16 * mo + 4 * g);
      s += from_bf16(w3[0]) * round_bf16(fmaxf(z[0] + b2.x, 0.0f));
      s += from_bf16(w3[1]) * round_bf16(fmaxf(z[1] + b2.y, 0.0f));
      s += from_bf16(w3[2]) * round_bf16(fmaxf(z[2] + b2.z, 0.0f));
      s += from_bf16(w3[3]) * round_bf16(fmaxf(z[3] + b2.w, 0.0f));
    }
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (g == nt) y = s;  // this lane's own sample is 16 nt + l%16 = l
  }
  return y + w.b3[0];
}

// The same products and sums as mlp_wave_forward_fast, in an order that loads
// every weight once per call: layer 1 for all four sample groups first, then
// each output tile's layer-2 weights serve the four groups.  Needs about 100
// more registers; for kernels that have them (the seed pass).
__device__ __forceinline__ float mlp_wave_forward_hoisted(const MlpDev &w, float x0, float x1, int l) {
  typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
  const int g = l >> 4, c = l & 15;
  bf16x8 bx = {0, 0, 0, 0, 0, 0, 0, 0};
  bx[0] = to_bf16(x0);
  bx[1] = to_bf16(x1);
  bf16x8 b2op[4][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const short w1a = w.w1b[2 * (16 * mt + c)], w1c = w.w1b[2 * (16 * mt + c) + 1];
    const float4 b1 = *(const float4 *)(w.b1 + 16 * mt + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      bf16x8 a1 = {0, 0, 0, 0, 0, 0, 0, 0};
      if (g == nt) {
        a1[0] = w1a;
        a1[1] = w1c;
      }
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bx, z, 0, 0, 0);
      b2op[nt][mt >> 1][4 * (mt & 1) + 0] = to_bf16(fmaxf(z[0] + b1.x, 0.0f));
      b2op[nt][mt >> 1][4 * (mt & 1) + 1] = to_bf16(fmaxf(z[1] + b1.y, 0.0f));
      b2op[nt][mt >> 1][4 * (mt & 1) + 2] = to_bf16(fmaxf(z[2] + b1.z, 0.0f));
      b2op[nt][mt >> 1][4 * (mt & 1) + 3] = to_bf16(fmaxf(z[3] + b1.w, 0.0f));
    }
  }
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int mo = 0; mo < 4; ++mo) {
    bf16x8 a2[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const short *row = w.w2b + (16 * mo + c) * H + 32 * kt + 4 * g;
      const bf16x4 lo = *(const bf16x4 *)row, hi = *(const bf16x4 *)(row + 16);
      a2[kt] = bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
    const float4 b2 = *(const float4 *)(w.b2 + 16 * mo + 4 * g);
    const bf16x4 w3 = *(const bf16x4 *)(w.w3b + 16 * mo + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[0], b2op[nt][0], z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[1], b2op[nt][1], z, 0, 0, 0);
      s[nt] += from_bf16(w3[0]) * round_bf16(fmaxf(z[0] + b2.x, 0.0f));
      s[nt] += from_bf16(w3[1]) * round_bf16(fmaxf(z[1] + b2.y, 0.0f));
      s[nt] += from_bf16(w3[2]) * round_bf16(fmaxf(z[2] + b2.z, 0.0f));
      s[nt] += from_bf16(w3[3]) * round_bf16(fmaxf(z[3] + b2.w, 0.0f));
    }
  }
  float y = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    float t = s[nt];
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    if (g == nt) y = t;
  }
  return y + w.b3[0];
}

__device__ __forceinline__ float norm01(double v, double lo, double hi) {
  return (float)(2.0 * (v - lo) / (hi - lo) - 1.0);
}

}  // namespace tdh
