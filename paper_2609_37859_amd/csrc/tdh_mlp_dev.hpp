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
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (short)(u >> 16);
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

// The same forward pass (bit for bit) with a lean register footprint, for use
// inside a larger kernel: one 16-sample tile at a time, and the lane index
// passed in (an opaque per-item value keeps the weight loads next to their
// use instead of hoisted into registers for the kernel's lifetime).
__device__ __forceinline__ float mlp_wave_forward_lean(const MlpDev &w, float x0, float x1, int l) {
  const float xb0 = round_bf16(x0), xb1 = round_bf16(x1);
  bf16x8 bop[4][2];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
      bop[nt][kt] = *(const bf16x8 *)(w.w2b + (16 * nt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
  const int src = 16 * ((l & 15) >> 2);
  float y = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int q = 16 * mt + (l & 15);
    const float q0 = __shfl(xb0, q, 64), q1 = __shfl(xb1, q, 64);
    bf16x8 a[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kt + 8 * (l >> 4) + e;
        float z = w.b1[k];
        z += from_bf16(w.w1b[2 * k]) * q0;
        z += from_bf16(w.w1b[2 * k + 1]) * q1;
        a[kt][e] = to_bf16(fmaxf(z, 0.0f));
      }
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bop[nt][0], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bop[nt][1], c, 0, 0, 0);
      acc[nt] = c;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int o = 16 * nt + (l & 15);
        const float h = round_bf16(fmaxf(acc[nt][r] + w.b2[o], 0.0f));
        s += from_bf16(w.w3b[o]) * h;
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      const float v = __shfl(s, src, 64);
      if (mt == (l >> 4) && r == (l & 3)) y = v;
    }
  }
  return y + w.b3[0];
}

__device__ __forceinline__ float norm01(double v, double lo, double hi) {
  return (float)(2.0 * (v - lo) / (hi - lo) - 1.0);
}

}  // namespace tdh
