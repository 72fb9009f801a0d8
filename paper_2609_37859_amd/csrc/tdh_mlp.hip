// Learned EOS seed: a 2 -> 64 -> 64 -> 1 ReLU network predicting normalised
// log T from normalised (log rho, log e), used to seed the table inversion.
// bf16 operands, fp32 accumulation.  The 64x64 hidden layer runs on the
// matrix cores (v_mfma_f32_16x16x32_bf16); the 2-wide input layer and the
// 1-wide output layer are plain vector arithmetic.
//
// MFMA 16x16x32 lane layout (lane l, e = 0..7, r = 0..3):
//   A (16 x 32, rows M):  row l%16, k = 8*(l/16) + e
//   B (32 x 16, cols N):  col l%16, k = 8*(l/16) + e
//   D (16 x 16):          col l%16, row 4*(l/16) + r
// A wave handles 64 samples: M/N tiles mt, nt in 0..3, K tiles kt in 0..1.
//
// Parameter vector (fp32 master copy, 4417 values): W1[64][2], b1[64],
// W2[64 out][64 in], b2[64], W3[64], b3.
#include "tdh_mlp_dev.hpp"

namespace tdh {

// ---------------------------------------------------------------------------
// inference over n queries (raw log10 rho, log10 e) -> log10 T
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpDev w, Seed s, const double *in, double *out,
                                                          long long n) {
  const long long nw = ((n + 63) / 64);
  const long long wave0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const long long wstride = ((long long)gridDim.x * blockDim.x) / 64;
  const int l = threadIdx.x & 63;
  for (long long wv = wave0; wv < nw; wv += wstride) {  // wave-uniform loop
    const long long q = wv * 64 + l;
    const bool ok = q < n;
    const float x0 = ok ? norm01(in[2 * q], s.lr_lo, s.lr_hi) : 0.0f;
    const float x1 = ok ? norm01(in[2 * q + 1], s.le_lo, s.le_hi) : 0.0f;
    const float y = mlp_wave_forward_fast(w, x0, x1, l);
    if (ok) out[q] = s.lt_lo + 0.5 * ((double)y + 1.0) * (s.lt_hi - s.lt_lo);
  }
}

// ---------------------------------------------------------------------------
// training: forward + backward of 64 samples per workgroup (one wave)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// sel: sample index per batch slot (nullptr: slot i -> sample i).
// part: per-workgroup gradient partials [gridDim.x][NPARAM]; loss_part[gridDim.x].
__global__ __launch_bounds__(64) void mlp_fwd_bwd_kernel(MlpDev w, Seed s, const double *in, const double *tgt,
                                                         long long n, int batch, uint64_t seed, int step,
                                                         int random_batch, float *part, float *loss_part) {
  __shared__ short h1[H * H];    // [q][k]
  __shared__ short h1t[H * H];   // [k][q]
  __shared__ short dz2[H * H];   // [q][o]
  __shared__ short dz2t[H * H];  // [o][q]
  const int l = threadIdx.x;
  const long long slot = (long long)blockIdx.x * 64 + l;
  long long q;
  if (random_batch)
    q = (long long)(splitmix64(seed ^ ((uint64_t)step << 32) ^ (uint64_t)slot) % (uint64_t)n);
  else
    q = slot;
  const float x0 = norm01(in[2 * q], s.lr_lo, s.lr_hi);
  const float x1 = norm01(in[2 * q + 1], s.le_lo, s.le_hi);
  const float t = norm01(tgt[q], s.lt_lo, s.lt_hi);
  const float xb0 = round_bf16(x0), xb1 = round_bf16(x1);
  // forward
  bf16x8 a[4][2];
  layer1_A(w, xb0, xb1, a);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const int qq = 16 * mt + (l & 15);
      const int k0 = 32 * kt + 8 * (l >> 4);
      *(bf16x8 *)(h1 + qq * H + k0) = a[mt][kt];
#pragma unroll
      for (int e = 0; e < 8; ++e) h1t[(k0 + e) * H + qq] = a[mt][kt][e];
    }
  f32x4 acc[4][4];
  layer2(w, a, acc);
  const float y = layer3(w, acc);
  const float dy = 2.0f * (y - t) / (float)batch;
  float loss = (y - t) * (y - t);
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  // output layer and hidden-layer gradients in D layout
  float gW3[4] = {0, 0, 0, 0}, gB2[4] = {0, 0, 0, 0};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int qq = 16 * mt + 4 * (l >> 4) + r;
      const float dyq = __shfl(dy, qq, 64);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int o = 16 * nt + (l & 15);
        const float z = acc[mt][nt][r] + w.b2[o];
        const float h = round_bf16(fmaxf(z, 0.0f));
        gW3[nt] += dyq * h;
        const float dz = z > 0.0f ? dyq * from_bf16(w.w3b[o]) : 0.0f;
        gB2[nt] += dz;
        const short db = to_bf16(dz);
        dz2[qq * H + o] = db;
        dz2t[o * H + qq] = db;
      }
    }
  __syncthreads();
  // dW2 = dz2^T h1: M = o, N = k, K = q
  float *P = part + (long long)blockIdx.x * NPARAM;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        const bf16x8 A = *(const bf16x8 *)(dz2t + (16 * mt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
        const bf16x8 B = *(const bf16x8 *)(h1t + (16 * nt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) P[OFF_W2 + (16 * mt + 4 * (l >> 4) + r) * H + 16 * nt + (l & 15)] = c[r];
    }
  // dH1 = dz2 W2: M = q, N = k, K = o; then the input layer
  float gB1[4] = {0, 0, 0, 0}, gW10[4] = {0, 0, 0, 0}, gW11[4] = {0, 0, 0, 0};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 c[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      c[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        const bf16x8 A = *(const bf16x8 *)(dz2 + (16 * mt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
        const bf16x8 B = *(const bf16x8 *)(w.w2tb + (16 * nt + (l & 15)) * H + 32 * kt + 8 * (l >> 4));
        c[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, c[nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int qq = 16 * mt + 4 * (l >> 4) + r;
      const float xq0 = __shfl(xb0, qq, 64), xq1 = __shfl(xb1, qq, 64);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int k = 16 * nt + (l & 15);
        float z1 = w.b1[k];
        z1 += from_bf16(w.w1b[2 * k]) * xq0;
        z1 += from_bf16(w.w1b[2 * k + 1]) * xq1;
        const float dz1 = z1 > 0.0f ? c[nt][r] : 0.0f;
        gB1[nt] += dz1;
        gW10[nt] += dz1 * xq0;
        gW11[nt] += dz1 * xq1;
      }
    }
  }
  // sum the per-lane partials over the four row groups (lanes with equal l%16)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    float v[5] = {gW3[nt], gB2[nt], gB1[nt], gW10[nt], gW11[nt]};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      v[i] += __shfl_xor(v[i], 16, 64);
      v[i] += __shfl_xor(v[i], 32, 64);
    }
    if (l < 16) {
      const int o = 16 * nt + l;
      P[OFF_W3 + o] = v[0];
      P[OFF_B2 + o] = v[1];
      P[OFF_B1 + o] = v[2];
      P[OFF_W1 + 2 * o] = v[3];
      P[OFF_W1 + 2 * o + 1] = v[4];
    }
  }
  float gb3 = dy;
  for (int o = 32; o > 0; o >>= 1) gb3 += __shfl_xor(gb3, o, 64);
  if (l == 0) {
    P[OFF_B3] = gb3;
    loss_part[blockIdx.x] = loss;
  }
}

// deterministic sum of the workgroup partials
__global__ void mlp_reduce_kernel(const float *part, int nparts, float *grad, const float *loss_part, float *loss,
                                  int batch) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPARAM; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[(long long)p * NPARAM + i];
    grad[i] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += loss_part[p];
    *loss = s / (float)batch;
  }
}

// Adam on fp32 master weights, then refresh the bf16 operand copies
__global__ void mlp_adam_kernel(float *wm, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPARAM; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    wm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void mlp_pack_kernel(const float *wm, short *w1b, short *w2b, short *w2tb, short *w3b, float *b1, float *b2,
                                float *b3) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPARAM; i += gridDim.x * blockDim.x) {
    const float x = wm[i];
    if (i < OFF_B1) {
      w1b[i] = to_bf16(x);
    } else if (i < OFF_W2) {
      b1[i - OFF_B1] = x;
    } else if (i < OFF_B2) {
      const int j = i - OFF_W2, o = j / H, k = j % H;
      w2b[o * H + k] = to_bf16(x);
      w2tb[k * H + o] = to_bf16(x);
    } else if (i < OFF_W3) {
      b2[i - OFF_B2] = x;
    } else if (i < OFF_B3) {
      w3b[i - OFF_W3] = to_bf16(x);
    } else {
      b3[0] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t mlp_launch_forward(const MlpDev &w, const Seed &s, const double *in, double *out, int64_t n,
                              hipStream_t st) {
  const long long waves = (n + 63) / 64;
  const long long blocks = (waves + 3) / 4;
  const int grid = blocks < 8192 ? (int)blocks : 8192;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, st, w, s, in, out, (long long)n);
  return hipGetLastError();
}

hipError_t mlp_launch_fwd_bwd(const MlpDev &w, const Seed &s, const double *in, const double *tgt, int64_t n,
                              int batch, uint64_t seed, int step, int random_batch, float *part, float *loss_part,
                              float *grad, float *loss, hipStream_t st) {
  hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3(batch / 64), dim3(64), 0, st, w, s, in, tgt, (long long)n, batch, seed,
                     step, random_batch, part, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, batch / 64, grad,
                     loss_part, loss, batch);
  return hipGetLastError();
}

hipError_t mlp_launch_adam(float *wm, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, wm, m, v, g, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

hipError_t mlp_launch_pack(const float *wm, short *w1b, short *w2b, short *w2tb, short *w3b, float *b1, float *b2,
                           float *b3, hipStream_t st) {
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, wm, w1b, w2b, w2tb, w3b, b1, b2,
                     b3);
  return hipGetLastError();
}

}  // namespace tdh
