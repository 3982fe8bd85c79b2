/*
 * mlp.c -- plain FP64 statement of the learned radiance cache (not in the
 * paper; an addition of this project).  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).
 *
 * Encoding (76 features): for axis a in (x, y, z) and k = 0..11,
 *   feats[24 a + 2 k] = sin(2^k pi p_a), feats[24 a + 2 k + 1] = cos(2^k pi p_a),
 * then the direction (3) and a normalised extinction (1); evaluated in FP64
 * and rounded once to FP32.
 * Network: 76 -> 64 -> 64 -> 64 -> 64 -> 3, ReLU after every hidden layer,
 * linear output.  Parameters: per layer W (row-major [out][in]) then b.
 * Loss: relative L2 (Mueller et al. 2021),
 *   loss = 1/(3B) sum (y - t)^2 / (stopgrad(y)^2 + 0.01).
 * Optimiser: Adam (Kingma & Ba 2015) with bias correction.
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

int oracle_nrc_encode(int64_t count, const float* pos, const float* dir, const float* sigma_norm, float* feats) {
  if (count < 0 || (count && (!pos || !dir || !sigma_norm || !feats))) return -1;
  const double pi = 3.14159265358979323846;
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
    f[75] = sigma_norm[i];
  }
  return 0;
}

/* Forward pass keeping every layer's pre-activation (z) and activation (a). */
static void forward_one(const double* P, const double* x, double acts[NLAYER + 1][NIN], double pre[NLAYER][NH]) {
  memcpy(acts[0], x, sizeof(double) * NIN);
  for (int l = 0; l < NLAYER; l++) {
    const double* W = P + layer_offset(l);
    const double* b = W + (int64_t)dims[l + 1] * dims[l];
    for (int o = 0; o < dims[l + 1]; o++) {
      double s = b[o];
      for (int i = 0; i < dims[l]; i++) s += W[(int64_t)o * dims[l] + i] * acts[l][i];
      pre[l][o] = s;
      acts[l + 1][o] = (l < NLAYER - 1) ? (s > 0.0 ? s : 0.0) : s;
    }
  }
}

int oracle_mlp_forward(const double* params, int64_t count, const double* x, double* y) {
  if (!params || count < 0 || (count && (!x || !y))) return -1;
  double acts[NLAYER + 1][NIN];
  double pre[NLAYER][NH];
  for (int64_t n = 0; n < count; n++) {
    forward_one(params, x + NIN * n, acts, pre);
    for (int c = 0; c < NOUT; c++) y[NOUT * n + c] = acts[NLAYER][c];
  }
  return 0;
}

/* Gradients of sum_n dy_n . y_n with respect to the parameters (summed over
 * the batch); also returns y. */
int oracle_mlp_backward(const double* params, int64_t count, const double* x, const double* dy, double* y,
                        double* grads) {
  if (!params || !grads || count < 0 || (count && (!x || !dy))) return -1;
  int64_t np = layer_offset(NLAYER);
  memset(grads, 0, sizeof(double) * (size_t)np);
  double acts[NLAYER + 1][NIN];
  double pre[NLAYER][NH];
  double delta[NIN], nd[NIN];
  for (int64_t n = 0; n < count; n++) {
    forward_one(params, x + NIN * n, acts, pre);
    if (y)
      for (int c = 0; c < NOUT; c++) y[NOUT * n + c] = acts[NLAYER][c];
    for (int c = 0; c < NOUT; c++) delta[c] = dy[NOUT * n + c]; /* linear output */
    for (int l = NLAYER - 1; l >= 0; l--) {
      const double* W = params + layer_offset(l);
      double* gW = grads + layer_offset(l);
      double* gb = gW + (int64_t)dims[l + 1] * dims[l];
      for (int o = 0; o < dims[l + 1]; o++) {
        gb[o] += delta[o];
        for (int i = 0; i < dims[l]; i++) gW[(int64_t)o * dims[l] + i] += delta[o] * acts[l][i];
      }
      if (l == 0) break;
      for (int i = 0; i < dims[l]; i++) {
        double s = 0.0;
        for (int o = 0; o < dims[l + 1]; o++) s += W[(int64_t)o * dims[l] + i] * delta[o];
        nd[i] = pre[l - 1][i] > 0.0 ? s : 0.0; /* ReLU derivative */
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
