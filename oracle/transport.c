/*
 * transport.c -- plain CPU statement of the volumetric path tracer
 * ("Volumetric Path Tracing" section of the paper: Algorithm 1 and "Path
 * Tracing within Tetrahedral Grids").  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).
 *
 * Algorithm 1 intersects the ray with the grid, then, while inside, reads
 * the density, samples a free path, marches through cells and samples the
 * phase function.  Readings of what it leaves open:
 *   - the free path is an optical depth tau ~ Exp(1) carried across cells
 *     (equal in distribution to per-cell resampling, by memorylessness);
 *   - inside a cell of extinction sigma and majorant sb >= sigma, tentative
 *     collisions come at rate sb (delta tracking); a tentative collision is
 *     real with probability sigma / sb (always real when sigma == sb, and
 *     then no extra number is drawn);
 *   - the phase function (Henyey-Greenstein) is sampled only at real
 *     collisions; the throughput is multiplied by the albedo there;
 *   - lights: one directional light (next-event estimation at every real
 *     collision, with transmittance to the boundary) and a constant
 *     environment added when the path leaves the grid; a camera ray that
 *     misses the grid sees the environment;
 *   - a path stops after max_bounces real collisions (after the light
 *     estimate at the last one); there is no Russian roulette;
 *   - extra channels (the paper's implementation carries e.g. temperature,
 *     albedo and phase-function parameters per tet; it gives no formulas).
 *     Reading: with channels on, a real collision in tet c first adds the
 *     emitted radiance by the collision estimator, beta * (1 - a_c) * T_c *
 *     emission (the absorbed fraction of the collision, FP32 in this order),
 *     then uses the tet's albedo a_c and phase parameter g_c in place of the
 *     medium's for the throughput, the light estimate and the phase sample.
 *     Absent channels keep the medium's values (temperature: no emission).
 *   - density models inside a tet (leb.c item 9, an extension): the tet's
 *     majorant comes from the model and each tentative collision evaluates
 *     the extinction at its point; the analytic light transmittance of the
 *     linear model integrates it exactly per segment (trapezoid rule).
 * Cell marching (at most four ray/face tests per cell in the paper; stored
 * normals let the direction rule faces out, leaving at most 3): for a face
 * with outward normal n (entries -1, 0, 1) and offset o_f,
 *   den = (n.x d.x + n.y d.y) + n.z d.z,  only den > 0 can be an exit,
 *   num = o_f 2^-20 - ((n.x o.x + n.y o.y) + n.z o.z),  t = num / den,
 * num and den in FP32 in exactly this order; the exit face is the one with
 * the smallest exact quotient num / den (lowest face index on ties; the
 * comparison num_f den_g < num_g den_f is exact in FP64), and the exit
 * distance is the correctly rounded FP32 quotient of that face, never less
 * than the current t.  (Rounding is monotone, so this distance is also the
 * minimum of the rounded quotients; only the choice between faces whose
 * quotients round to the same float is made exactly.)
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 * seed, counter = (pixel, sample, (bounce << 8) | stream, draw >> 2), word
 * draw & 3; u = (word >> 8) * 2^-24.  Streams: 0 camera, 1 free flight,
 * 2 phase, 3 light transmittance.  "bounce" = number of real collisions so
 * far.  Arithmetic is FP32 except the exact FP64 comparison of exit
 * quotients and the transcendentals (FP64 library functions on the FP32
 * argument, rounded once to FP32).
 */
#include "oracle_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

enum { ST_CAMERA = 0, ST_FLIGHT = 1, ST_PHASE = 2, ST_NEE = 3 };

/* ---------------- Philox4x32-10 ---------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

float oracle_uniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t stream,
                     uint32_t draw) {
  uint32_t ctr[4] = {pixel, sample, (bounce << 8) | stream, draw >> 2};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return (float)(out[draw & 3] >> 8) * 0x1p-24f;
}

typedef struct {
  uint64_t seed;
  uint32_t pixel, sample;
  uint32_t bounce;
  uint32_t draws[4]; /* per stream, reset at every bounce */
} rng_t;

static float rnd(rng_t* r, int stream) {
  return oracle_uniform(r->seed, r->pixel, r->sample, r->bounce, (uint32_t)stream, r->draws[stream]++);
}

/* ---------------- elementary functions ----------------
 * Every transcendental of the method is taken at its plain definition: the
 * FP64 C library function evaluated on the FP32 argument (exact in FP64) and
 * rounded once to FP32.  A device implementation that meets the same
 * definition to within an FP32 ulp or so reproduces the oracle's paths except
 * where a comparison sits within that ulp. */
float oracle_neglog1m(float u) { return (float)(0.0 - log1p(-(double)u)); }

float oracle_expneg(float x) { return (float)exp(-(double)x); }

void oracle_sincos2pi(float u, float* c, float* s) {
  double a = (2.0 * OR_PI) * (double)u;
  *c = (float)cos(a);
  *s = (float)sin(a);
}

/* Exponential optical depth from a uniform (inversion of the Exp(1) CDF). */
static float sample_tau(float u) { return oracle_neglog1m(u); }

/* ---------------- Henyey-Greenstein ---------------- */
/* p(mu) = (1 - g^2) / (4 pi (1 + g^2 - 2 g mu)^(3/2)), mu = cosine between
 * successive propagation directions; FP64, rounded once. */
float oracle_hg_eval(float g, float mu) {
  double gg = (double)g, m = (double)mu;
  double g2 = gg * gg;
  double den = (1.0 + g2) - (2.0 * gg) * m;
  return (float)((1.0 - g2) / (((4.0 * OR_PI) * den) * sqrt(den)));
}

/* Inversion of the HG cumulative distribution (mu increasing in u); for
 * |g| < 1e-3 its g -> 0 limit, the isotropic 2u - 1.  FP64, clamped to
 * [-1, 1], rounded once. */
float oracle_hg_sample_mu(float g, float u) {
  double gg = (double)g, uu = (double)u, mu;
  if (fabs(gg) < 1e-3) {
    mu = 2.0 * uu - 1.0;
  } else {
    double g2 = gg * gg;
    double sv = (1.0 - g2) / ((1.0 - gg) + (2.0 * gg) * uu);
    mu = ((1.0 + g2) - sv * sv) / (2.0 * gg);
  }
  if (mu < -1.0) mu = -1.0;
  if (mu > 1.0) mu = 1.0;
  return (float)mu;
}

static void normalize3f(float v[3]) {
  float l = sqrtf((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
  v[0] = v[0] / l;
  v[1] = v[1] / l;
  v[2] = v[2] / l;
}

/* New direction: mu from HG, azimuth 2 pi u2, in the orthonormal basis of
 * Duff et al. (2017) around d. */
void oracle_hg_direction(const float d[3], float g, float u1, float u2, float out[3]) {
  float mu = oracle_hg_sample_mu(g, u1);
  float q = 1.0f - mu * mu;
  if (q < 0.0f) q = 0.0f;
  float st = sqrtf(q);
  float cp, sp;
  oracle_sincos2pi(u2, &cp, &sp);
  float sign = copysignf(1.0f, d[2]);
  float a = -1.0f / (sign + d[2]);
  float b = (d[0] * d[1]) * a;
  float t1[3] = {1.0f + ((sign * d[0]) * d[0]) * a, sign * b, -sign * d[0]};
  float t2[3] = {b, sign + (d[1] * d[1]) * a, -d[1]};
  float ca = st * cp, cb = st * sp;
  for (int i = 0; i < 3; i++) out[i] = (t1[i] * ca + t2[i] * cb) + d[i] * mu;
  normalize3f(out);
}

/* ---------------- camera ---------------- */
typedef struct {
  float pos[3], f[3], r[3], u[3];
  float tan_x, tan_y;
  int32_t w, h;
} frame32;

static void make_frame(const ocam* k, frame32* fr) {
  double pos[3], f[3], r[3], u[3], up[3];
  for (int i = 0; i < 3; i++) {
    pos[i] = (double)k->pos[i];
    f[i] = (double)k->look_at[i] - pos[i];
    up[i] = (double)k->up[i];
  }
  double l = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
  for (int i = 0; i < 3; i++) f[i] = f[i] / l;
  r[0] = f[1] * up[2] - f[2] * up[1];
  r[1] = f[2] * up[0] - f[0] * up[2];
  r[2] = f[0] * up[1] - f[1] * up[0];
  l = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
  for (int i = 0; i < 3; i++) r[i] = r[i] / l;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  double tan_y = tan((double)k->fov_y_deg * (OR_PI / 360.0));
  double tan_x = tan_y * (double)k->width / (double)k->height;
  for (int i = 0; i < 3; i++) {
    fr->pos[i] = k->pos[i];
    fr->f[i] = (float)f[i];
    fr->r[i] = (float)r[i];
    fr->u[i] = (float)u[i];
  }
  fr->tan_x = (float)tan_x;
  fr->tan_y = (float)tan_y;
  fr->w = k->width;
  fr->h = k->height;
}

static void frame_ray(const frame32* fr, int32_t px, int32_t py, float u0, float u1, float o[3], float d[3]) {
  float sx = ((2.0f * (((float)px + u0) / (float)fr->w)) - 1.0f) * fr->tan_x;
  float sy = (1.0f - 2.0f * (((float)py + u1) / (float)fr->h)) * fr->tan_y;
  for (int i = 0; i < 3; i++) {
    o[i] = fr->pos[i];
    d[i] = (fr->f[i] + sx * fr->r[i]) + sy * fr->u[i];
  }
  normalize3f(d);
}

void oracle_camera_ray(const ocam* cam, int32_t px, int32_t py, float u0, float u1, float o[3], float d[3]) {
  frame32 fr;
  make_frame(cam, &fr);
  frame_ray(&fr, px, py, u0, u1, o, d);
}

/* Ray against the unit cube; returns 1 and the entry point on a hit.  The
 * entry point is clamped to [0,1] and its entering coordinate set exactly to
 * the face value when the origin is outside. */
static int enter_cube(const float o[3], const float d[3], float p[3]) {
  float tn = -INFINITY, tf = INFINITY;
  int axis = -1;
  for (int a = 0; a < 3; a++) {
    if (d[a] == 0.0f) {
      if (o[a] < 0.0f || o[a] > 1.0f) return 0;
      continue;
    }
    float inv = 1.0f / d[a];
    float ta = (0.0f - o[a]) * inv, tb = (1.0f - o[a]) * inv;
    float lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
    if (lo > tn) {
      tn = lo;
      axis = a;
    }
    if (hi < tf) tf = hi;
  }
  if (tn > tf || tf <= 0.0f) return 0;
  float te = tn > 0.0f ? tn : 0.0f;
  for (int a = 0; a < 3; a++) {
    float v = o[a] + te * d[a];
    if (v < 0.0f) v = 0.0f;
    if (v > 1.0f) v = 1.0f;
    p[a] = v;
  }
  if (tn > 0.0f && axis >= 0) p[axis] = d[axis] > 0.0f ? 0.0f : 1.0f;
  return 1;
}

/* ---------------- media: tet grid or voxel grid ---------------- */
typedef struct {
  int kind; /* 0 tets, 1 voxels */
  const ogrid* g;
  const float* dens;
  int32_t n;
  float scale;
} medium_t;

/* Exit of cell `cell` along (o, d) from parameter t (face rule in the file
 * header).  Returns the exit face
 * (tets: 0..3, voxels: axis 0..2) or -1, with *te the exit parameter and
 * *next the next cell (-1 = leaves the grid). */
static int cell_exit(const medium_t* m, int64_t cell, const float o[3], const float d[3], float t, float* te,
                     int64_t* next) {
  if (m->kind == 0) {
    const ogrid* g = m->g;
    int best = -1;
    float bnum = 0.0f, bden = 1.0f;
    for (int f = 0; f < 4; f++) {
      int code = g->codes[4 * cell + f];
      const int32_t* dir = or_dirs[code >> 1];
      float s = (code & 1) ? -1.0f : 1.0f;
      float n0 = s * (float)dir[0], n1 = s * (float)dir[1], n2 = s * (float)dir[2];
      float den = (n0 * d[0] + n1 * d[1]) + n2 * d[2];
      if (!(den > 0.0f)) continue;
      float num = ldexpf((float)g->offsets[4 * cell + f], -OR_LAT_BITS) - ((n0 * o[0] + n1 * o[1]) + n2 * o[2]);
      /* exact comparison of num/den with the best so far: FP64 products of
       * FP32 values are exact */
      if (best < 0 || (double)num * (double)bden < (double)bnum * (double)den) {
        best = f;
        bnum = num;
        bden = den;
      }
    }
    if (best < 0) return -1;
    float bt = bnum / bden;
    *te = bt > t ? bt : t;
    uint32_t nb = g->nbr[4 * cell + best];
    *next = nb == OR_BOUNDARY ? -1 : (int64_t)(nb >> 2);
    return best;
  } else {
    int64_t n = m->n;
    int64_t idx[3] = {cell % n, (cell / n) % n, cell / (n * n)};
    int best = -1;
    float bt = 0.0f;
    for (int a = 0; a < 3; a++) {
      if (d[a] == 0.0f) continue;
      float plane = d[a] > 0.0f ? (float)(idx[a] + 1) / (float)n : (float)idx[a] / (float)n;
      float tf = (plane - o[a]) / d[a];
      if (best < 0 || tf < bt) {
        best = a;
        bt = tf;
      }
    }
    if (best < 0) return -1;
    *te = bt > t ? bt : t;
    idx[best] += d[best] > 0.0f ? 1 : -1;
    if (idx[best] < 0 || idx[best] >= n)
      *next = -1;
    else
      *next = idx[0] + n * (idx[1] + n * idx[2]);
    return best;
  }
}

static float cell_sigma(const medium_t* m, int64_t cell) {
  return m->kind == 0 ? m->g->sigma[cell] : m->scale * m->dens[cell];
}

static float cell_majorant(const medium_t* m, int64_t cell) {
  return m->kind == 0 ? m->g->majorant[cell] : m->scale * m->dens[cell];
}

/* Density models (leb.c item 9).  With a model on, a tet's majorant is the
 * model's and the extinction is evaluated at each tentative collision point
 * x (FP32): model 1 ((c0 + gx x) + gy y) + gz z, model 2 the scale times
 * the voxel floor(x n) (indices clamped to the volume). */
static int has_model(const medium_t* m) { return m->kind == 0 && m->g->model != 0; }

static float model_majorant(const medium_t* m, int64_t cell) {
  return has_model(m) ? m->g->mmaj[cell] : cell_majorant(m, cell);
}

static float point_sigma(const medium_t* m, int64_t cell, const float x[3]) {
  const ogrid* g = m->g;
  if (g->model == 1) {
    const float* c = g->mcoef + 4 * cell;
    return ((c[0] + c[1] * x[0]) + c[2] * x[1]) + c[3] * x[2];
  }
  int64_t n = g->mn, idx[3];
  for (int a = 0; a < 3; a++) {
    int64_t i = (int64_t)floorf(x[a] * (float)n);
    idx[a] = i < 0 ? 0 : (i >= n ? n - 1 : i);
  }
  return g->mscale * g->mdens[idx[0] + n * (idx[1] + n * idx[2])];
}

static int64_t locate_cell(const medium_t* m, const float p[3]) {
  if (m->kind == 0) return or_locate_point(m->g, p);
  int64_t idx[3];
  for (int a = 0; a < 3; a++) {
    int64_t i = (int64_t)floorf(p[a] * (float)m->n);
    if (i < 0) i = 0;
    if (i >= m->n) i = m->n - 1;
    idx[a] = i;
  }
  return idx[0] + m->n * (idx[1] + m->n * idx[2]);
}

/* ---------------- path ---------------- */
typedef struct {
  int64_t steps; /* exit evaluations of this path (all walks) */
  int64_t max_steps;
  orender_stats* st;
} budget_t;

/* Transmittance from x along w to the boundary, starting in `cell`.
 * mode 0: exp(-sum sigma_i dt_i); 1: ratio tracking against the majorant;
 * 2: delta tracking (0 or 1).  Returns -1 when the step budget runs out. */
static float shadow(const medium_t* m, int64_t cell, const float x[3], const float w[3], int mode, rng_t* rng,
                    budget_t* b) {
  float t = 0.0f, od = 0.0f, tr = 1.0f;
  float tau = 0.0f;
  if (mode != 0) tau = sample_tau(rnd(rng, ST_NEE));
  for (;;) {
    if (b->steps >= b->max_steps) return -1.0f;
    float te;
    int64_t next;
    int f = cell_exit(m, cell, x, w, t, &te, &next);
    b->steps++;
    b->st->tet_steps++;
    if (f < 0) break;
    if (mode == 0 && has_model(m)) {
      /* linear model: the exact integral of a linear function over the
       * segment, its length times the mean of the end values */
      float xa[3], xb[3];
      for (int i = 0; i < 3; i++) {
        xa[i] = x[i] + t * w[i];
        xb[i] = x[i] + te * w[i];
      }
      od = od + (0.5f * (point_sigma(m, cell, xa) + point_sigma(m, cell, xb))) * (te - t);
    } else if (mode == 0) {
      od = od + cell_sigma(m, cell) * (te - t);
    } else {
      float s = cell_sigma(m, cell), sb = model_majorant(m, cell);
      if (sb > 0.0f) {
        float dtau = sb * (te - t);
        while (tau < dtau) {
          t = t + tau / sb;
          if (has_model(m)) {
            float xt[3];
            for (int i = 0; i < 3; i++) xt[i] = x[i] + t * w[i];
            s = point_sigma(m, cell, xt);
          }
          if (mode == 1) {
            tr = tr * (1.0f - s / sb);
          } else {
            int real = 1;
            if (s < sb) real = rnd(rng, ST_NEE) < s / sb;
            if (real) return 0.0f;
          }
          tau = sample_tau(rnd(rng, ST_NEE));
          dtau = sb * (te - t);
        }
        tau = tau - dtau;
      }
      if (mode == 1 && tr == 0.0f) return 0.0f;
    }
    t = te;
    if (next < 0) break;
    cell = next;
  }
  if (mode == 0) return oracle_expneg(od);
  return tr;
}

/* Radiance cache hooks of a path (NULL: the plain estimator).
 *   truncate > 0: at real vertex `truncate` the path adds the cache's
 *     estimate times the throughput reaching the vertex (before the albedo)
 *     and stops; there is no light estimate at that vertex (the cache covers
 *     it).
 *   rec != NULL: vertices 1..max_rec are recorded, 11 floats each: the
 *     vertex x (3), the incoming direction d (3), the extinction at the
 *     vertex, the throughput reaching the vertex, and L gathered before it
 *     (3); *n_rec = number recorded.
 * The extinction at a vertex, the cache's input there, is the cell's; on a
 * grid with a density model, the model's at the vertex.  With channels the
 * cache at vertex k stands for the vertex's own emission too (records are
 * taken before it). */
typedef struct {
  int32_t truncate;
  const double* params;
  int32_t bf16;
  float sigma_ref;
  int32_t max_rec;
} nrc_hook;

static void trace_path(const medium_t* m, const frame32* fr, const omedium* med, const olight* lt,
                       const orender_opts* op, uint64_t seed, int32_t px, int32_t py, uint32_t sample, float L[3],
                       orender_stats* st, const nrc_hook* hk, float* rec, int32_t* n_rec) {
  rng_t rng;
  memset(&rng, 0, sizeof(rng));
  rng.seed = seed;
  rng.pixel = (uint32_t)(py * fr->w + px);
  rng.sample = sample;
  float o[3], d[3], p[3];
  float u0 = rnd(&rng, ST_CAMERA), u1 = rnd(&rng, ST_CAMERA);
  frame_ray(fr, px, py, u0, u1, o, d);
  L[0] = L[1] = L[2] = 0.0f;
  if (!enter_cube(o, d, p)) {
    for (int c = 0; c < 3; c++) L[c] = lt->env_radiance[c];
    return;
  }
  int64_t cell = locate_cell(m, p);
  if (cell < 0) {
    for (int c = 0; c < 3; c++) L[c] = lt->env_radiance[c];
    return;
  }
  memcpy(o, p, sizeof(o));
  float t = 0.0f;
  float beta[3] = {1.0f, 1.0f, 1.0f};
  float tau = sample_tau(rnd(&rng, ST_FLIGHT));
  budget_t b = {0, op->max_steps_per_path, st};
  for (;;) {
    if (b.steps >= b.max_steps) {
      st->truncated++;
      return;
    }
    float te;
    int64_t next;
    int f = cell_exit(m, cell, o, d, t, &te, &next);
    b.steps++;
    st->tet_steps++;
    if (f < 0) { /* no exit face: leave the grid */
      for (int c = 0; c < 3; c++) L[c] = L[c] + beta[c] * lt->env_radiance[c];
      st->escapes++;
      return;
    }
    float s = cell_sigma(m, cell), sb = model_majorant(m, cell);
    int collided = 0;
    float tc = 0.0f;
    if (sb > 0.0f) {
      float dtau = sb * (te - t);
      while (tau < dtau) {
        tc = t + tau / sb;
        if (has_model(m)) { /* the extinction at the tentative collision */
          float xt[3];
          for (int i = 0; i < 3; i++) xt[i] = o[i] + tc * d[i];
          s = point_sigma(m, cell, xt);
        }
        int real = 1;
        if (s < sb) real = rnd(&rng, ST_FLIGHT) < s / sb;
        if (real) {
          collided = 1;
          break;
        }
        st->null_collisions++;
        t = tc;
        tau = sample_tau(rnd(&rng, ST_FLIGHT));
        dtau = sb * (te - t);
      }
      if (!collided) tau = tau - dtau;
    }
    if (collided) {
      st->real_collisions++;
      float x[3];
      for (int i = 0; i < 3; i++) x[i] = o[i] + tc * d[i];
      rng.bounce++;
      memset(rng.draws, 0, sizeof(rng.draws));
      /* s: the extinction at the collision (the tet's, or the density
       * model's at the point), the cache's input there */
      if (hk && hk->truncate == (int32_t)rng.bounce) {
        float r[3];
        oracle_nrc_eval_point(hk->params, hk->bf16, hk->sigma_ref, x, d, s, r);
        for (int c = 0; c < 3; c++) L[c] = L[c] + beta[c] * r[c];
        return;
      }
      if (rec && (int32_t)rng.bounce <= hk->max_rec) {
        float* q = rec + 11 * (rng.bounce - 1);
        for (int i = 0; i < 3; i++) {
          q[i] = x[i];
          q[3 + i] = d[i];
          q[8 + i] = L[i];
        }
        q[6] = s;
        q[7] = beta[0];
        *n_rec = (int32_t)rng.bounce;
      }
      /* extra channels of the collision's tet: emission (absorbed part of
       * the collision: (1 - albedo) * temperature * emission colour, the
       * collision estimator of the emitted radiance), then its albedo and
       * phase parameter in place of the medium's */
      float alb = med->albedo, gg = med->g;
      if (op->channels) {
        const ogrid* gr = m->g;
        if (gr->ch[1]) alb = gr->ch[1][cell];
        if (gr->ch[2]) gg = gr->ch[2][cell];
        if (gr->ch[0]) {
          float e = (1.0f - alb) * gr->ch[0][cell];
          for (int c = 0; c < 3; c++) L[c] = L[c] + beta[c] * (e * op->emission[c]);
        }
      }
      for (int c = 0; c < 3; c++) beta[c] = beta[c] * alb;
      float tr = shadow(m, cell, x, lt->sun_dir, op->transmittance, &rng, &b);
      if (tr < 0.0f) {
        st->truncated++;
        return;
      }
      float mu = (d[0] * lt->sun_dir[0] + d[1] * lt->sun_dir[1]) + d[2] * lt->sun_dir[2];
      float ph = oracle_hg_eval(gg, mu);
      for (int c = 0; c < 3; c++) L[c] = L[c] + ((beta[c] * ph) * lt->sun_irradiance[c]) * tr;
      if ((int32_t)rng.bounce >= op->max_bounces) return;
      float v1 = rnd(&rng, ST_PHASE), v2 = rnd(&rng, ST_PHASE);
      float nd[3];
      oracle_hg_direction(d, gg, v1, v2, nd);
      memcpy(d, nd, sizeof(d));
      memcpy(o, x, sizeof(o));
      t = 0.0f;
      tau = sample_tau(rnd(&rng, ST_FLIGHT));
      continue;
    }
    t = te;
    if (next < 0) {
      for (int c = 0; c < 3; c++) L[c] = L[c] + beta[c] * lt->env_radiance[c];
      st->escapes++;
      return;
    }
    cell = next;
  }
}

static int check_render_args(const ocam* cam, const omedium* med, const olight* lt, int32_t spp,
                             const orender_opts* op, const int32_t* pixels, int64_t n_pixels, float* out) {
  if (!cam || !med || !lt || !op || !out || spp < 1 || n_pixels < 0) return -1;
  if (cam->width < 1 || cam->height < 1 || !(cam->fov_y_deg > 0.0f && cam->fov_y_deg < 180.0f)) return -1;
  if (op->max_bounces < 1 || op->transmittance < 0 || op->transmittance > 2 || op->max_steps_per_path < 1 ||
      op->sample_offset < 0)
    return -1;
  if (!(med->g > -1.0f && med->g < 1.0f) || !(med->albedo >= 0.0f)) return -1;
  if (pixels)
    for (int64_t i = 0; i < n_pixels; i++)
      if (pixels[i] < 0 || (int64_t)pixels[i] >= (int64_t)cam->width * cam->height) return -1;
  return 0;
}

/* Channels need a tet grid that carries at least one of them and a finite,
 * non-negative emission colour.  They combine with the radiance cache: the
 * cache at vertex k stands for all radiance from k on, the vertex's own
 * emission included (the record of vertex k is taken before it). */
static int check_channels(const medium_t* m, const orender_opts* op) {
  if (!op->channels) return 0;
  if (m->kind != 0 || (!m->g->ch[0] && !m->g->ch[1] && !m->g->ch[2])) return -1;
  for (int c = 0; c < 3; c++)
    if (!(op->emission[c] >= 0.0f) || isinf(op->emission[c])) return -1;
  return 0;
}

static int render_common(const medium_t* m, const ocam* cam, const omedium* med, const olight* lt, int32_t spp,
                         uint64_t seed, const orender_opts* op, const int32_t* pixels, int64_t n_pixels,
                         float* out, orender_stats* stats, int32_t threads, const nrc_hook* hk) {
  int rc = check_render_args(cam, med, lt, spp, op, pixels, pixels ? n_pixels : 0, out);
  if (rc) return rc;
  if (has_model(m) && m->g->model == 2 && op->transmittance == 0) return -1; /* voxel lookups: no analytic light */
  if (check_channels(m, op)) return -1;
  frame32 fr;
  make_frame(cam, &fr);
  int64_t np = pixels ? n_pixels : (int64_t)cam->width * cam->height;
  orender_stats tot;
  memset(&tot, 0, sizeof(tot));
  int nt = threads > 1 ? threads : 1;
  (void)nt;
  int64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt) reduction(+ : a0, a1, a2, a3, a4)
  for (int64_t i = 0; i < np; i++) {
    int64_t pix = pixels ? pixels[i] : i;
    int32_t px = (int32_t)(pix % cam->width), py = (int32_t)(pix / cam->width);
    orender_stats st;
    memset(&st, 0, sizeof(st));
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int32_t s = 0; s < spp; s++) {
      float L[3];
      trace_path(m, &fr, med, lt, op, seed, px, py, (uint32_t)(op->sample_offset + s), L, &st, hk, NULL,
                 NULL);
      for (int c = 0; c < 3; c++) acc[c] = acc[c] + L[c];
    }
    for (int c = 0; c < 3; c++) out[3 * i + c] = acc[c] / (float)spp;
    a0 += st.tet_steps;
    a1 += st.null_collisions;
    a2 += st.real_collisions;
    a3 += st.escapes;
    a4 += st.truncated;
  }
  if (stats) {
    stats->tet_steps = a0;
    stats->null_collisions = a1;
    stats->real_collisions = a2;
    stats->escapes = a3;
    stats->truncated = a4;
  }
  return 0;
}

int oracle_tet_render(const ogrid* g, const ocam* cam, const omedium* med, const olight* light, int32_t spp,
                      uint64_t seed, const orender_opts* opts, const int32_t* pixels, int64_t n_pixels,
                      float* out_rgb, orender_stats* stats, int32_t threads) {
  if (!g) return -1;
  medium_t m = {0, g, NULL, 0, 1.0f};
  return render_common(&m, cam, med, light, spp, seed, opts, pixels, n_pixels, out_rgb, stats, threads, NULL);
}

int oracle_dda_render(const float* density, int32_t n, float density_scale, const ocam* cam, const omedium* med,
                      const olight* light, int32_t spp, uint64_t seed, const orender_opts* opts,
                      const int32_t* pixels, int64_t n_pixels, float* out_rgb, orender_stats* stats,
                      int32_t threads) {
  if (!density || n < 1 || (n & (n - 1))) return -1;
  medium_t m = {1, NULL, density, n, density_scale};
  return render_common(&m, cam, med, light, spp, seed, opts, pixels, n_pixels, out_rgb, stats, threads, NULL);
}

int oracle_walk(const ogrid* g, const float o[3], const float d[3], int64_t start, int32_t max_out, int64_t* tets,
                int32_t* faces, float* texit, int32_t* n_out) {
  if (!g || !o || !d || start < 0 || start >= g->n || max_out < 1 || !tets || !faces || !texit || !n_out)
    return -1;
  medium_t m = {0, g, NULL, 0, 1.0f};
  int64_t cell = start;
  float t = 0.0f;
  int32_t k = 0;
  while (k < max_out) {
    float te;
    int64_t next;
    int f = cell_exit(&m, cell, o, d, t, &te, &next);
    tets[k] = cell;
    faces[k] = f;
    texit[k] = te;
    k++;
    if (f < 0 || next < 0) break;
    t = te;
    cell = next;
  }
  *n_out = k;
  return 0;
}

/* ---------------- radiance cache (not in the paper) ----------------
 * Truncated render: every path stops at real vertex truncate_bounce, adding
 * the throughput reaching it times the cache's estimate there. */
int oracle_nrc_render(const ogrid* g, const ocam* cam, const omedium* med, const olight* light, int32_t spp,
                      uint64_t seed, const orender_opts* opts, const double* params, int32_t bf16,
                      int32_t truncate_bounce, float sigma_ref, const int32_t* pixels, int64_t n_pixels,
                      float* out_rgb, orender_stats* stats, int32_t threads) {
  if (!g || !params || truncate_bounce < 1 || !(sigma_ref > 0.0f)) return -1;
  medium_t m = {0, g, NULL, 0, 1.0f};
  nrc_hook hk = {truncate_bounce, params, bf16, sigma_ref, 0};
  return render_common(&m, cam, med, light, spp, seed, opts, pixels, n_pixels, out_rgb, stats, threads, &hk);
}

/* Pixel of training path j: a 24-bit uniform integer w (from the draw of
 * stream 4 with counter pixel = j, sample 0, bounce 0) scaled to the image,
 * floor(w * npix / 2^24). */
int32_t oracle_train_pixel(uint64_t frame_seed, uint32_t j, int64_t npix) {
  float u = oracle_uniform(frame_seed, j, 0, 0, 4, 0);
  uint64_t w = (uint64_t)(u * 16777216.0f);
  return (int32_t)((w * (uint64_t)npix) >> 24);
}

/* Training records of one frame: path j (0 <= j < n_paths) is the plain
 * estimator's sample j of pixel oracle_train_pixel(frame_seed, j) with seed
 * frame_seed, never truncated.  Its vertices k = 1..max_vertices with a
 * positive throughput give one record each, in (path, vertex) order: the
 * vertex, the incoming direction, the cell's extinction and the target
 * (L_final - L_before_k) / beta_k (FP32, per channel), where beta_k is the
 * throughput reaching vertex k (before its albedo) and L_before_k the
 * radiance gathered before it; tag = 16 j + (k - 1).  Arrays hold
 * n_paths * max_vertices records; path_pixel and path_L (n_paths and
 * 3 n_paths, may be NULL) receive each path's pixel and final radiance. */
int oracle_nrc_collect(const ogrid* g, const ocam* cam, const omedium* med, const olight* light, uint64_t frame_seed,
                       const orender_opts* opts, int32_t n_paths, int32_t max_vertices, float* pos, float* dir,
                       float* sigma, float* target, int32_t* tag, int64_t* count, int32_t* path_pixel, float* path_L,
                       int32_t threads) {
  if (!g || n_paths < 0 || n_paths > (1 << 26) || max_vertices < 1 || max_vertices > 16 || !pos || !dir || !sigma ||
      !target || !tag || !count)
    return -1;
  int rc = check_render_args(cam, med, light, 1, opts, NULL, 0, target);
  if (rc) return rc;
  medium_t m = {0, g, NULL, 0, 1.0f};
  if (check_channels(&m, opts)) return -1;
  if (g->model == 2 && opts->transmittance == 0) return -1;
  frame32 fr;
  make_frame(cam, &fr);
  int64_t npix = (int64_t)cam->width * cam->height;
  float* rec = (float*)malloc(sizeof(float) * 11 * (size_t)max_vertices * (size_t)(n_paths ? n_paths : 1));
  int32_t* nv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_paths ? n_paths : 1));
  float* Lf = (float*)malloc(sizeof(float) * 3 * (size_t)(n_paths ? n_paths : 1));
  if (!rec || !nv || !Lf) {
    free(rec);
    free(nv);
    free(Lf);
    return -2;
  }
  nrc_hook hk = {0, NULL, 0, 0.0f, max_vertices};
  int nt = threads > 1 ? threads : 1;
  (void)nt;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
  for (int32_t j = 0; j < n_paths; j++) {
    int32_t pix = oracle_train_pixel(frame_seed, (uint32_t)j, npix);
    orender_stats st;
    memset(&st, 0, sizeof(st));
    nv[j] = 0;
    trace_path(&m, &fr, med, light, opts, frame_seed, (int32_t)(pix % cam->width), (int32_t)(pix / cam->width),
               (uint32_t)j, Lf + 3 * (size_t)j, &st, &hk, rec + 11 * (size_t)max_vertices * (size_t)j, nv + j);
    if (path_pixel) path_pixel[j] = pix;
  }
  int64_t c = 0;
  for (int32_t j = 0; j < n_paths; j++) {
    for (int32_t k = 0; k < nv[j]; k++) {
      const float* q = rec + 11 * ((size_t)max_vertices * (size_t)j + (size_t)k);
      if (!(q[7] > 0.0f)) continue;
      for (int i = 0; i < 3; i++) {
        pos[3 * c + i] = q[i];
        dir[3 * c + i] = q[3 + i];
        target[3 * c + i] = (Lf[3 * j + i] - q[8 + i]) / q[7];
      }
      sigma[c] = q[6];
      tag[c] = 16 * j + k;
      c++;
    }
    if (path_L)
      for (int i = 0; i < 3; i++) path_L[3 * j + i] = Lf[3 * j + i];
  }
  *count = c;
  free(rec);
  free(nv);
  free(Lf);
  return 0;
}
