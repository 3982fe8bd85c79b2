/*
 * gen.c -- seeded synthetic density volumes standing in for the paper's
 * OpenVDB assets (a cloud, an explosion), which are not available.  Holds no
 * part of the rendering method; both the oracle and the GPU path consume its
 * output as plain input.
 *
 * Voxel (i, j, k) of an n^3 grid covers [i/n, (i+1)/n) x ... of the unit
 * cube and is stored at index i + n (j + n k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double u01(uint64_t* s) { return (double)(sm64(s) >> 11) * 0x1p-53; }

/* Sum of isotropic Gaussian blobs evaluated in FP64 at voxel centres:
 * centres U[0.2,0.8]^3, std-devs U[0.05,0.2], peaks U[2,10]. */
void synth_blobs(uint64_t seed, int32_t n, int32_t nblobs, float* out) {
  uint64_t s = seed * 0x2545F4914F6CDD1Dull + 1;
  double c[64][3], r[64], pk[64];
  if (nblobs > 64) nblobs = 64;
  for (int b = 0; b < nblobs; b++) {
    for (int a = 0; a < 3; a++) c[b][a] = 0.2 + 0.6 * u01(&s);
    r[b] = 0.05 + 0.15 * u01(&s);
    pk[b] = 2.0 + 8.0 * u01(&s);
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++)
    for (int64_t j = 0; j < n; j++)
      for (int64_t i = 0; i < n; i++) {
        double p[3] = {(i + 0.5) / n, (j + 0.5) / n, (k + 0.5) / n};
        double v = 0.0;
        for (int b = 0; b < nblobs; b++) {
          double d2 = 0.0;
          for (int a = 0; a < 3; a++) d2 += (p[a] - c[b][a]) * (p[a] - c[b][a]);
          v += pk[b] * exp(-d2 / (2.0 * r[b] * r[b]));
        }
        out[i + n * (j + n * k)] = (float)v;
      }
}

/* ---------------- gradient noise (Perlin 2002 style) ---------------- */
static const double grad12[12][3] = {{1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 0, 1}, {-1, 0, 1},
                                     {1, 0, -1}, {-1, 0, -1}, {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

static uint32_t lattice_hash(int64_t x, int64_t y, int64_t z, uint64_t seed) {
  uint64_t h = seed ^ ((uint64_t)x * 0x8DA6B343ull) ^ ((uint64_t)y * 0xD8163841ull) ^ ((uint64_t)z * 0xCB1AB31Full);
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 32;
  return (uint32_t)h;
}

static double fade(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }

static double gnoise(double x, double y, double z, uint64_t seed) {
  double fx = floor(x), fy = floor(y), fz = floor(z);
  int64_t ix = (int64_t)fx, iy = (int64_t)fy, iz = (int64_t)fz;
  double dx = x - fx, dy = y - fy, dz = z - fz;
  double v[8];
  for (int q = 0; q < 8; q++) {
    int a = q & 1, b = (q >> 1) & 1, c = (q >> 2) & 1;
    const double* g = grad12[lattice_hash(ix + a, iy + b, iz + c, seed) % 12];
    v[q] = g[0] * (dx - a) + g[1] * (dy - b) + g[2] * (dz - c);
  }
  double u = fade(dx), w = fade(dy), t = fade(dz);
  double x00 = v[0] + u * (v[1] - v[0]), x10 = v[2] + u * (v[3] - v[2]);
  double x01 = v[4] + u * (v[5] - v[4]), x11 = v[6] + u * (v[7] - v[6]);
  double y0 = x00 + w * (x10 - x00), y1 = x01 + w * (x11 - x01);
  return y0 + t * (y1 - y0);
}

static double fbm(double x, double y, double z, int octaves, double freq, uint64_t seed) {
  double s = 0.0, amp = 1.0, norm = 0.0;
  for (int o = 0; o < octaves; o++) {
    s += amp * gnoise(x * freq, y * freq, z * freq, seed + 0x9E37ull * (uint64_t)o);
    norm += amp;
    amp *= 0.5;
    freq *= 2.0;
  }
  return s / norm;
}

/* Un-thresholded cloud field: 6-octave fBm (lacunarity 2, gain 0.5, base
 * frequency 4) times a smooth ellipsoidal falloff; >= 0. */
void synth_cloud_raw(uint64_t seed, int32_t n, float* out) {
  const double rad[3] = {0.42, 0.30, 0.38};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n; k++)
    for (int64_t j = 0; j < n; j++)
      for (int64_t i = 0; i < n; i++) {
        double p[3] = {(i + 0.5) / n, (j + 0.5) / n, (k + 0.5) / n};
        double q = 0.0;
        for (int a = 0; a < 3; a++) q += ((p[a] - 0.5) / rad[a]) * ((p[a] - 0.5) / rad[a]);
        double fall = q < 1.0 ? (1.0 - q) * (1.0 - q) : 0.0;
        double v = 0.0;
        if (fall > 0.0) v = (0.5 + 0.7 * fbm(p[0], p[1], p[2], 6, 4.0, seed)) * fall;
        out[i + n * (j + n * k)] = (float)(v > 0.0 ? v : 0.0);
      }
}

/* Smoke-plume field: fBm sampled at points advected backwards along a
 * divergence-free (curl of a noise potential) velocity for 4 steps, inside
 * a Gaussian radial mask widening with height, times exp(-h / H). */
static void curl(double x, double y, double z, uint64_t seed, double v[3]) {
  /* the potential's components are three decorrelated noises; central
   * differences give its curl */
  const double e = 1e-3;
  double dpz_dy = (gnoise(x, y + e, z, seed + 3) - gnoise(x, y - e, z, seed + 3)) / (2 * e);
  double dpy_dz = (gnoise(x, y, z + e, seed + 2) - gnoise(x, y, z - e, seed + 2)) / (2 * e);
  double dpx_dz = (gnoise(x, y, z + e, seed + 1) - gnoise(x, y, z - e, seed + 1)) / (2 * e);
  double dpz_dx = (gnoise(x + e, y, z, seed + 3) - gnoise(x - e, y, z, seed + 3)) / (2 * e);
  double dpy_dx = (gnoise(x + e, y, z, seed + 2) - gnoise(x - e, y, z, seed + 2)) / (2 * e);
  double dpx_dy = (gnoise(x, y + e, z, seed + 1) - gnoise(x, y - e, z, seed + 1)) / (2 * e);
  v[0] = dpz_dy - dpy_dz;
  v[1] = dpx_dz - dpz_dx;
  v[2] = dpy_dx - dpx_dy;
}

/* The advection map p -> q(p) is smooth (the curl field's features span a
 * third of the domain), so it is sampled on a lattice of 129^3 points over
 * [0,1]^3 and interpolated trilinearly at the voxel centres. */
#define PLUME_L 129
void synth_plume_raw(uint64_t seed, int32_t n, float* out) {
  const int64_t L = PLUME_L;
  double* Q = (double*)malloc(sizeof(double) * 3 * (size_t)(L * L * L));
  if (!Q) return;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < L; k++)
    for (int64_t j = 0; j < L; j++)
      for (int64_t i = 0; i < L; i++) {
        double q[3] = {3.0 * i / (L - 1), 3.0 * j / (L - 1), 3.0 * k / (L - 1)};
        for (int s = 0; s < 4; s++) {
          double c[3];
          curl(q[0], q[1], q[2], seed, c);
          for (int a = 0; a < 3; a++) q[a] -= 0.06 * c[a];
        }
        for (int a = 0; a < 3; a++) Q[3 * (i + L * (j + L * k)) + a] = q[a];
      }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n; k++)
    for (int64_t j = 0; j < n; j++)
      for (int64_t i = 0; i < n; i++) {
        double p[3] = {(i + 0.5) / n, (j + 0.5) / n, (k + 0.5) / n};
        double h = p[1];
        double rr = 0.06 + 0.25 * h;
        double dx = p[0] - 0.5, dz = p[2] - 0.5;
        double mask = exp(-(dx * dx + dz * dz) / (2.0 * rr * rr)) * exp(-h / 0.45);
        double v = 0.0;
        if (mask > 1e-3) {
          double g[3], f[3];
          int64_t c0[3];
          for (int a = 0; a < 3; a++) {
            g[a] = p[a] * (L - 1);
            c0[a] = (int64_t)g[a];
            if (c0[a] > L - 2) c0[a] = L - 2;
            f[a] = g[a] - c0[a];
          }
          double q[3] = {0.0, 0.0, 0.0};
          for (int c = 0; c < 8; c++) {
            int64_t ci = c0[0] + (c & 1), cj = c0[1] + ((c >> 1) & 1), ck = c0[2] + ((c >> 2) & 1);
            double w = ((c & 1) ? f[0] : 1.0 - f[0]) * (((c >> 1) & 1) ? f[1] : 1.0 - f[1]) *
                       (((c >> 2) & 1) ? f[2] : 1.0 - f[2]);
            const double* qq = Q + 3 * (ci + L * (cj + L * ck));
            for (int a = 0; a < 3; a++) q[a] += w * qq[a];
          }
          v = (0.5 + 0.8 * fbm(q[0] / 3.0, q[1] / 3.0 - 0.2 * h, q[2] / 3.0, 5, 6.0, seed + 77)) * mask;
        }
        out[i + n * (j + n * k)] = (float)(v > 0.0 ? v : 0.0);
      }
  free(Q);
}

/* In place: v = max(v - cut, 0) * (float)(peak / max), cut = the value of
 * rank floor((1 - keep_fraction) count) in ascending order (exact radix
 * selection on the bit patterns of these non-negative floats: upper 16
 * bits, then lower 16 bits). */
void synth_threshold(float* v, int64_t count, double keep_fraction, double peak) {
  int64_t rank = (int64_t)((1.0 - keep_fraction) * (double)count);
  if (rank >= count) rank = count - 1;
  uint64_t* hist = (uint64_t*)calloc(65536, sizeof(uint64_t));
  if (!hist) return;
  uint32_t prefix = 0;
  for (int pass = 0; pass < 2; pass++) {
    memset(hist, 0, 65536 * sizeof(uint64_t));
#pragma omp parallel
    {
      uint64_t* h = (uint64_t*)calloc(65536, sizeof(uint64_t));
#pragma omp for schedule(static)
      for (int64_t i = 0; i < count; i++) {
        uint32_t u;
        memcpy(&u, v + i, 4);
        if (pass == 0) h[u >> 16]++;
        else if ((u >> 16) == prefix) h[u & 0xFFFFu]++;
      }
#pragma omp critical
      for (int b = 0; b < 65536; b++) hist[b] += h[b];
      free(h);
    }
    int b = 0;
    while (rank >= (int64_t)hist[b]) {
      rank -= (int64_t)hist[b];
      b++;
    }
    prefix = pass == 0 ? (uint32_t)b : ((prefix << 16) | (uint32_t)b);
  }
  free(hist);
  float cut;
  memcpy(&cut, &prefix, 4);
  float m = 0.0f;
#pragma omp parallel for reduction(max : m)
  for (int64_t i = 0; i < count; i++) {
    float d = v[i] - cut;
    v[i] = d > 0.0f ? d : 0.0f;
    m = v[i] > m ? v[i] : m;
  }
  if (m > 0.0f) {
    float sc = (float)(peak / (double)m);
#pragma omp parallel for
    for (int64_t i = 0; i < count; i++) v[i] = v[i] * sc;
  }
}
