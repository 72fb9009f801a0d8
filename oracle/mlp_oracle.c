/*
 * FP64 oracle of the learned EOS seed: a 2 -> 64 -> 64 -> 1 ReLU network
 * mapping normalised (log rho, log e) to normalised log T, trained with a
 * mean-squared-error loss and Adam.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).
 *
 * With round_bf16 = 1 the operands of every matrix product (inputs,
 * weights, hidden activations, and the back-propagated pre-activation
 * gradients) are rounded to bfloat16 (round to nearest even, taken from the
 * float32 value), as the GPU kernels do; accumulation is FP64 here.  With
 * round_bf16 = 0 the network is the plain FP64 function, whose gradient is
 * checked against finite differences.  Weight gradients are taken with
 * respect to the rounded weights that were used (straight-through).
 *
 * Parameter vector (4417 doubles): W1[64][2], b1[64], W2[64][64] (row =
 * output unit), b2[64], W3[64], b3.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + 2 * H)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)
#define NPARAM (OFF_B3 + 1)

static double bf16r(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double rnd(double x, int r) { return r ? bf16r(x) : x; }

typedef struct {
  double xr[2], z1[H], h1r[H], z2[H], h2r[H], y;
} fwd_t;

static void forward_one(const double *p, int r, const double *x, fwd_t *f) {
  f->xr[0] = rnd(x[0], r);
  f->xr[1] = rnd(x[1], r);
  for (int o = 0; o < H; o++) {
    double z = p[OFF_B1 + o];
    z += rnd(p[OFF_W1 + 2 * o], r) * f->xr[0];
    z += rnd(p[OFF_W1 + 2 * o + 1], r) * f->xr[1];
    f->z1[o] = z;
    f->h1r[o] = rnd(z > 0.0 ? z : 0.0, r);
  }
  for (int o = 0; o < H; o++) {
    double z = p[OFF_B2 + o];
    for (int q = 0; q < H; q++) z += rnd(p[OFF_W2 + H * o + q], r) * f->h1r[q];
    f->z2[o] = z;
    f->h2r[o] = rnd(z > 0.0 ? z : 0.0, r);
  }
  double y = p[OFF_B3];
  for (int o = 0; o < H; o++) y += rnd(p[OFF_W3 + o], r) * f->h2r[o];
  f->y = y;
}

void orc_mlp_forward(const double *p, int r, int64_t n, const double *x, double *y) {
  for (int64_t s = 0; s < n; s++) {
    fwd_t f;
    forward_one(p, r, x + 2 * s, &f);
    y[s] = f.y;
  }
}

/* mean squared error and its gradient over n samples; returns the loss */
double orc_mlp_loss_grad(const double *p, int r, int64_t n, const double *x, const double *t, double *g) {
  memset(g, 0, NPARAM * sizeof(double));
  double loss = 0.0;
  for (int64_t s = 0; s < n; s++) {
    fwd_t f;
    forward_one(p, r, x + 2 * s, &f);
    double e = f.y - t[s];
    loss += e * e;
    double dy = 2.0 * e / (double)n;
    g[OFF_B3] += dy;
    double dz2r[H], dz1[H];
    for (int o = 0; o < H; o++) {
      g[OFF_W3 + o] += dy * f.h2r[o];
      double dz2 = f.z2[o] > 0.0 ? dy * rnd(p[OFF_W3 + o], r) : 0.0;
      g[OFF_B2 + o] += dz2;
      dz2r[o] = rnd(dz2, r);
    }
    for (int o = 0; o < H; o++)
      for (int q = 0; q < H; q++) g[OFF_W2 + H * o + q] += dz2r[o] * f.h1r[q];
    for (int q = 0; q < H; q++) {
      double dh = 0.0;
      for (int o = 0; o < H; o++) dh += rnd(p[OFF_W2 + H * o + q], r) * dz2r[o];
      dz1[q] = f.z1[q] > 0.0 ? dh : 0.0;
      g[OFF_B1 + q] += dz1[q];
      g[OFF_W1 + 2 * q] += dz1[q] * f.xr[0];
      g[OFF_W1 + 2 * q + 1] += dz1[q] * f.xr[1];
    }
  }
  return loss / (double)n;
}

/* one Adam step (Kingma & Ba) on master weights */
void orc_mlp_adam(double *w, double *m, double *v, const double *g, int step, double lr, double b1, double b2,
                  double eps, int64_t n) {
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int64_t i = 0; i < n; i++) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}
