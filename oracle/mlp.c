/*
 * mlp.c -- plain FP64 statement of the learned radiance cache (not in the
 * paper; an addition of this project, after Mueller et al. 2021, "Real-time
 * Neural Radiance Caching for Path Tracing").  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).
 *
 * Encoding (76 features) of a point p, a direction d and the extinction
 * sigma of the cell holding p: for axis a in (x, y, z) and k = 0..11,
 *   feats[24 a + 2 k] = sin(2^k pi p_a), feats[24 a + 2 k + 1] = cos(2^k pi p_a),
 * then d (3) and log(1 + sigma) / log(1 + sigma_ref) (1); evaluated in FP64
 * and rounded once to FP32.
 * Network: 76 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU after every hidden layer,
 * linear output.  Parameters: per layer W (row-major [out][in]) then b.
 * Loss: relative L2 (Mueller et al. 2021),
 *   loss = 1/(3B) sum (y - t)^2 / (stopgrad(y)^2 + 0.01).
 * Optimiser: Adam (Kingma & Ba 2015) with bias correction.  Inference may use
 * an exponential moving average of the weights after each step, bias
 * corrected like Adam's moments: ema_t = b ema_{t-1} + (1 - b) w_t, ema_0 = 0,
 * weights = ema_t / (1 - b^t).
 *
 * BF16-operand mode (bf16 != 0) states the precision the GPU network runs
 * in: every operand of a matrix product is rounded to bfloat16 (round to
 * nearest even, from its FP32 value) before the product, and products are
 * summed exactly (here: in FP64).  The operands are the weights, each
 * layer's input (the features, then the hidden activations) and, in the
 * backward pass, the back-propagated errors.  Biases, bias gradients,
 * pre-activations and the loss stay in wide precision.  The ReLU derivative
 * is 1 where the rounded activation is positive.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NIN 76
#define NH 64
#define NOUT 3
#define NLAYER 5

static const int dims[NLAYER + 1] = {NIN, NH, NH, NH, NH, NOUT};

static int64_t layer_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; i++) o += (int64_t)dims[i + 1] * dims[i] + dims[i + 1];
  return o;
}

/* bfloat16 = the upper 16 bits of an FP32 word; rounding to nearest, ties
 * to even, on the discarded lower 16 bits.  NaN stays NaN. */
float oracle_bf16_round(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
    u |= 0x00400000u; /* quiet NaN */
    u &= 0xFFFF0000u;
  } else {
    uint32_t low = u & 0xFFFFu, keep = u >> 16;
    if (low > 0x8000u || (low == 0x8000u && (keep & 1u))) keep += 1u; /* may carry into the exponent */
    u = keep << 16;
  }
  float r;
  memcpy(&r, &u, 4);
  return r;
}

static double q16(double v) { return (double)oracle_bf16_round((float)v); }

int oracle_nrc_encode(int64_t count, const float* pos, const float* dir, const float* sigma, float sigma_ref,
                      float* feats) {
  if (count < 0 || (count && (!pos || !dir || !sigma || !feats)) || !(sigma_ref > 0.0f)) return -1;
  const double pi = 3.14159265358979323846;
  const double lref = log1p((double)sigma_ref);
  for (int64_t i = 0; i < count; i++) {
    float* f = feats + NIN * i;
    for (int a = 0; a < 3; a++)
      for (int k = 0; k < 12; k++) {
        double arg = ((double)(1 << k) * pi) * (double)pos[3 * i + a];
        f[24 * a + 2 * k] = (float)sin(arg);
        f[24 * a + 2 * k + 1] = (float)cos(arg);
      }
    f[72] = dir[3 * i];
    f[73] = dir[3 * i + 1];
    f[74] = dir[3 * i + 2];
    if (!(sigma[i] >= 0.0f)) return -5;
    f[75] = (float)(log1p((double)sigma[i]) / lref);
  }
  return 0;
}

/* Forward pass keeping every layer's input (acts, as used by the product)
 * and pre-activation (pre). */
static void forward_one(const double* P, const double* x, int bf16, double acts[NLAYER + 1][NIN],
                        double pre[NLAYER][NH]) {
  for (int i = 0; i < NIN; i++) acts[0][i] = bf16 ? q16(x[i]) : x[i];
  for (int l = 0; l < NLAYER; l++) {
    const double* W = P + layer_offset(l);
    const double* b = W + (int64_t)dims[l + 1] * dims[l];
    for (int o = 0; o < dims[l + 1]; o++) {
      double s = 0.0;
      for (int i = 0; i < dims[l]; i++) {
        double w = W[(int64_t)o * dims[l] + i];
        s += (bf16 ? q16(w) : w) * acts[l][i];
      }
      s += b[o];
      pre[l][o] = s;
      if (l < NLAYER - 1) {
        double a = s > 0.0 ? s : 0.0;
        acts[l + 1][o] = bf16 ? q16(a) : a;
      } else {
        acts[l + 1][o] = s;
      }
    }
  }
}

int oracle_mlp_forward(const double* params, int64_t count, const double* x, double* y, int32_t bf16) {
  if (!params || count < 0 || (count && (!x || !y))) return -1;
  double acts[NLAYER + 1][NIN];
  double pre[NLAYER][NH];
  for (int64_t n = 0; n < count; n++) {
    forward_one(params, x + NIN * n, bf16, acts, pre);
    for (int c = 0; c < NOUT; c++) y[NOUT * n + c] = acts[NLAYER][c];
  }
  return 0;
}

/* Gradients of sum_n dy_n . y_n with respect to the parameters (summed over
 * the batch); also returns y. */
int oracle_mlp_backward(const double* params, int64_t count, const double* x, const double* dy, double* y,
                        double* grads, int32_t bf16) {
  if (!params || !grads || count < 0 || (count && (!x || !dy))) return -1;
  int64_t np = layer_offset(NLAYER);
  memset(grads, 0, sizeof(double) * (size_t)np);
  double acts[NLAYER + 1][NIN];
  double pre[NLAYER][NH];
  double delta[NIN], dq[NIN], nd[NIN];
  for (int64_t n = 0; n < count; n++) {
    forward_one(params, x + NIN * n, bf16, acts, pre);
    if (y)
      for (int c = 0; c < NOUT; c++) y[NOUT * n + c] = acts[NLAYER][c];
    for (int c = 0; c < NOUT; c++) delta[c] = dy[NOUT * n + c]; /* linear output */
    for (int l = NLAYER - 1; l >= 0; l--) {
      const double* W = params + layer_offset(l);
      double* gW = grads + layer_offset(l);
      double* gb = gW + (int64_t)dims[l + 1] * dims[l];
      for (int o = 0; o < dims[l + 1]; o++) dq[o] = bf16 ? q16(delta[o]) : delta[o];
      for (int o = 0; o < dims[l + 1]; o++) {
        gb[o] += delta[o];
        for (int i = 0; i < dims[l]; i++) gW[(int64_t)o * dims[l] + i] += dq[o] * acts[l][i];
      }
      if (l == 0) break;
      for (int i = 0; i < dims[l]; i++) {
        double s = 0.0;
        for (int o = 0; o < dims[l + 1]; o++) {
          double w = W[(int64_t)o * dims[l] + i];
          s += (bf16 ? q16(w) : w) * dq[o];
        }
        /* ReLU derivative: the unit was active (in BF16 mode: its rounded
         * activation, the value the next layer used, is positive) */
        int on = bf16 ? acts[l][i] > 0.0 : pre[l - 1][i] > 0.0;
        nd[i] = on ? s : 0.0;
      }
      memcpy(delta, nd, sizeof(double) * (size_t)dims[l]);
    }
  }
  return 0;
}

int oracle_nrc_loss_grad(int64_t count, const double* y, const double* target, double* loss, double* dy) {
  if (count < 1 || !y || !target) return -1;
  double s = 0.0;
  double norm = 1.0 / (3.0 * (double)count);
  for (int64_t i = 0; i < 3 * count; i++) {
    double den = y[i] * y[i] + 0.01;
    double e = y[i] - target[i];
    s += e * e / den;
    if (dy) dy[i] = 2.0 * e / den * norm;
  }
  if (loss) *loss = s * norm;
  return 0;
}

int oracle_adam_step(int64_t n, double* params, const double* grads, double* m, double* v, int64_t step, double lr,
                     double beta1, double beta2, double eps) {
  if (n < 0 || step < 1 || !params || !grads || !m || !v) return -1;
  double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  for (int64_t i = 0; i < n; i++) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grads[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grads[i] * grads[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    params[i] -= lr * mh / (sqrt(vh) + eps);
  }
  return 0;
}

int oracle_ema_step(int64_t n, double* ema, const double* params, double beta, int64_t step, double* out) {
  if (n < 0 || step < 1 || !ema || !params || !out || !(beta >= 0.0 && beta < 1.0)) return -1;
  double c = 1.0 - pow(beta, (double)step);
  for (int64_t i = 0; i < n; i++) {
    ema[i] = beta * ema[i] + (1.0 - beta) * params[i];
    out[i] = ema[i] / c;
  }
  return 0;
}

/* The cache's radiance estimate at one path vertex, as the truncated
 * render adds it: the network output clamped at zero, in FP32. */
void oracle_nrc_eval_point(const double* params, int32_t bf16, float sigma_ref, const float p[3], const float d[3],
                           float sigma, float out[3]) {
  float f[NIN];
  double x[NIN], acts[NLAYER + 1][NIN], pre[NLAYER][NH];
  oracle_nrc_encode(1, p, d, &sigma, sigma_ref, f);
  for (int i = 0; i < NIN; i++) x[i] = f[i];
  forward_one(params, x, bf16, acts, pre);
  for (int c = 0; c < NOUT; c++) {
    float v = (float)acts[NLAYER][c];
    out[c] = v > 0.0f ? v : 0.0f;
  }
}
