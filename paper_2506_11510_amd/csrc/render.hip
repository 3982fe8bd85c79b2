// render.hip -- Monte Carlo volumetric path tracing through the tet grid
// (paper, "Volumetric Path Tracing": Algorithm 1 and "Path Tracing within
// Tetrahedral Grids").
//
// One persistent kernel: every lane runs a small state machine over its own
// paths (fetch work -> camera ray, grid entry and point location -> walk
// steps of the main path -> walk steps of the light (shadow) ray -> ...).
// Each loop iteration advances every busy lane by one cell, so lanes whose
// paths have very different lengths stay busy; idle lanes take new work
// items from a device counter with one atomic per wave (ballot + popcount).
//
// One walk step reads one 48-byte tet record (face plane offsets, face
// normals in 6 bits each, 4 neighbour links, extinction, majorant) and
// evaluates only faces whose outward normal faces the ray (n.d > 0, at most
// 3), in FP32 in a fixed order; the free flight is delta tracking against the
// per-tet majorant with an optical depth carried across cells; real
// collisions scatter by Henyey-Greenstein after a next-event estimate of the
// directional light (transmittance by walking the light ray to the grid
// boundary); paths leaving the grid see the constant environment.
//
// The same kernel, instantiated on the voxel grid (Amanatides-Woo steps),
// is the regular-grid reference renderer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"

namespace tv {

struct RenderArgs {
  const TetRec* rec;
  const uint64_t* keys;
  int64_t n;
  int32_t dmax;
  const float* dens;  // voxel medium
  int32_t nvox;
  float scale;
  Frame fr;
  float albedo, g;
  float sun[3], E[3], env[3];
  int32_t spp, sample_offset, per_item, items_per_pixel, max_bounces, transmittance;
  int64_t max_steps;
  uint64_t seed;
  uint32_t items;
  int32_t tiles_x;
  float* out;
  uint32_t* counter;
  unsigned long long* stats;
  int accumulate;
};

struct Step {
  float te, sigma, majorant;
  int32_t next;  // -1: leaves the grid
  bool ok;       // false: no exit face
};

// ---------------------------------------------------------------- tet medium
template <int K>
__device__ inline void descend_point(int32_t v[4][3], uint64_t& h, const double P[3]) {
  constexpr int J1 = K == 1 ? 2 : 1, J2 = K == 3 ? 2 : 3;
  int32_t z[3];
  int64_t a[3], b[3], nn[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    z[i] = (v[0][i] + v[K][i]) >> 1;
    a[i] = (int64_t)v[J1][i] - z[i];
    b[i] = (int64_t)v[J2][i] - z[i];
  }
  nn[0] = a[1] * b[2] - a[2] * b[1];
  nn[1] = a[2] * b[0] - a[0] * b[2];
  nn[2] = a[0] * b[1] - a[1] * b[0];
  int64_t s0 = nn[0] * (v[0][0] - z[0]) + nn[1] * (v[0][1] - z[1]) + nn[2] * (v[0][2] - z[2]);
  double side = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    int sg = (nn[i] > 0) - (nn[i] < 0);
    if (s0 < 0) sg = -sg;
    if (sg) side = side + (double)sg * (P[i] - (double)z[i]);
  }
  if (side >= 0.0) {
#pragma unroll
    for (int i = 0; i < 3; i++) v[K][i] = z[i];
    h = 2 * h;
  } else {
#pragma unroll
    for (int j = 0; j < K; j++)
#pragma unroll
      for (int i = 0; i < 3; i++) v[j][i] = v[j + 1][i];
#pragma unroll
    for (int i = 0; i < 3; i++) v[K][i] = z[i];
    h = 2 * h + 1;
  }
}

// Tet containing p: the Kuhn root whose axis order sorts p's coordinates in
// descending order, exact bisection-plane descent to the grid's depth, then
// the last tet whose depth-first key is <= the key reached.
__device__ inline int64_t locate_point(const uint64_t* __restrict__ keys, int64_t n, int dmax, float3 p) {
  const float c[3] = {p.x, p.y, p.z};
  int r = -1;
  if (c[0] >= c[1] && c[1] >= c[2]) r = 0;
  else if (c[0] >= c[2] && c[2] >= c[1]) r = 1;
  else if (c[1] >= c[0] && c[0] >= c[2]) r = 2;
  else if (c[1] >= c[2] && c[2] >= c[0]) r = 3;
  else if (c[2] >= c[0] && c[0] >= c[1]) r = 4;
  else if (c[2] >= c[1] && c[1] >= c[0]) r = 5;
  if (r < 0) return -1;
  const int p0 = (r < 2) ? 0 : (r < 4 ? 1 : 2);
  const int p1 = (r == 0 || r == 5) ? 1 : ((r == 1 || r == 3) ? 2 : 0);
  int32_t v[4][3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    v[0][a] = 0;
    v[1][a] = a == p0 ? kLatS : 0;
    v[2][a] = (a == p0 || a == p1) ? kLatS : 0;
    v[3][a] = kLatS;
  }
  double P[3] = {(double)p.x * (double)kLatS, (double)p.y * (double)kLatS, (double)p.z * (double)kLatS};
  uint64_t h = 8 + (uint64_t)r;
  for (int d = 0; d < dmax; d += 3) {
    descend_point<3>(v, h, P);
    if (d + 1 < dmax) descend_point<2>(v, h, P);
    if (d + 2 < dmax) descend_point<1>(v, h, P);
  }
  uint64_t key = h << (60 - dmax);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (keys[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

struct TetMedium {
  const TetRec* __restrict__ rec;
  const uint64_t* __restrict__ keys;
  int64_t n;
  int dmax;
  __device__ inline int64_t locate(float3 p) const { return locate_point(keys, n, dmax, p); }
  __device__ inline Step step(uint32_t cell, float3 o, float3 d, float t) const {
    const float4* q = (const float4*)(rec + cell);
    float4 offs = q[0];
    uint4 nb = *(const uint4*)(q + 1);
    float4 w = q[2];
    uint32_t normals = __float_as_uint(w.x);
    const float off[4] = {offs.x, offs.y, offs.z, offs.w};
    int best = -1;
    float bt = 0.0f;
#pragma unroll
    for (int f = 0; f < 4; f++) {
      uint32_t c = (normals >> (6 * f)) & 63u;
      float nx = (float)((int)(c & 3u) - 1), ny = (float)((int)((c >> 2) & 3u) - 1),
            nz = (float)((int)((c >> 4) & 3u) - 1);
      float den = (nx * d.x + ny * d.y) + nz * d.z;
      if (den > 0.0f) {
        float num = off[f] - ((nx * o.x + ny * o.y) + nz * o.z);
        float tf = num / den;
        if (best < 0 || tf < bt) {
          best = f;
          bt = tf;
        }
      }
    }
    Step s;
    s.sigma = w.y;
    s.majorant = w.z;
    s.ok = best >= 0;
    s.te = bt > t ? bt : t;
    uint32_t link = best == 0 ? nb.x : (best == 1 ? nb.y : (best == 2 ? nb.z : nb.w));
    s.next = (!s.ok || link == kBoundary) ? -1 : (int32_t)(link >> 2);
    return s;
  }
};

// ---------------------------------------------------------------- voxel medium
struct VoxelMedium {
  const float* __restrict__ dens;
  int32_t n;
  float scale;
  __device__ inline int64_t locate(float3 p) const {
    float c[3] = {p.x, p.y, p.z};
    int64_t idx[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      int64_t i = (int64_t)floorf(c[a] * (float)n);
      idx[a] = i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    return idx[0] + n * (idx[1] + (int64_t)n * idx[2]);
  }
  __device__ inline Step step(uint32_t cell, float3 o, float3 d, float t) const {
    int32_t idx[3] = {(int32_t)(cell % (uint32_t)n), (int32_t)((cell / (uint32_t)n) % (uint32_t)n),
                      (int32_t)(cell / ((uint32_t)n * (uint32_t)n))};
    const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    int best = -1;
    float bt = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (dd[a] == 0.0f) continue;
      float plane = dd[a] > 0.0f ? (float)(idx[a] + 1) / (float)n : (float)idx[a] / (float)n;
      float tf = (plane - oo[a]) / dd[a];
      if (best < 0 || tf < bt) {
        best = a;
        bt = tf;
      }
    }
    Step s;
    float v = scale * dens[cell];
    s.sigma = v;
    s.majorant = v;
    s.ok = best >= 0;
    s.te = bt > t ? bt : t;
    s.next = -1;
    if (s.ok) {
      int32_t nx = idx[0], ny = idx[1], nz = idx[2];
      int32_t step = dd[best] > 0.0f ? 1 : -1;
      if (best == 0) nx += step;
      else if (best == 1) ny += step;
      else nz += step;
      if (nx >= 0 && nx < n && ny >= 0 && ny < n && nz >= 0 && nz < n)
        s.next = nx + n * (ny + n * nz);
    }
    return s;
  }
};

// ---------------------------------------------------------------- camera
__device__ inline bool enter_cube(float3 o, float3 d, float3& p) {
  const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
  float tn = -INFINITY, tf = INFINITY;
  int axis = -1;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (dd[a] == 0.0f) {
      if (oo[a] < 0.0f || oo[a] > 1.0f) return false;
      continue;
    }
    float inv = 1.0f / dd[a];
    float ta = (0.0f - oo[a]) * inv, tb = (1.0f - oo[a]) * inv;
    float lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
    if (lo > tn) {
      tn = lo;
      axis = a;
    }
    if (hi < tf) tf = hi;
  }
  if (tn > tf || tf <= 0.0f) return false;
  float te = tn > 0.0f ? tn : 0.0f;
  float r[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    float v = oo[a] + te * dd[a];
    v = v < 0.0f ? 0.0f : v;
    v = v > 1.0f ? 1.0f : v;
    r[a] = v;
  }
  if (tn > 0.0f && axis >= 0) {
    float fv = dd[axis] > 0.0f ? 0.0f : 1.0f;
    if (axis == 0) r[0] = fv;
    else if (axis == 1) r[1] = fv;
    else r[2] = fv;
  }
  p = make_float3(r[0], r[1], r[2]);
  return true;
}

// ---------------------------------------------------------------- kernel
enum { M_FETCH = 0, M_START = 1, M_TRACK = 2, M_SHADOW = 3, M_DONE = 4 };

template <class Med>
__global__ __launch_bounds__(256) void k_render(RenderArgs A, Med med) {
  const int lane = __lane_id();
  int mode = M_FETCH;
  uint32_t pix = 0;
  int32_t s = 0, s_end = 0;
  float3 o = make_float3(0, 0, 0), d = o, dsave = o, beta = o, L = o, acc = o;
  float t = 0.0f, tau = 0.0f, od = 0.0f, tr = 1.0f;
  uint32_t cell = 0, cell_x = 0, bounce = 0, jf = 0, jn = 0;
  int64_t steps = 0;
  unsigned long long c_steps = 0;
  uint32_t c_null = 0, c_real = 0, c_esc = 0, c_trunc = 0;
  const float3 sun = make_float3(A.sun[0], A.sun[1], A.sun[2]);

  for (;;) {
    // ---- idle lanes take work items (one atomic per wave)
    bool need = mode == M_FETCH;
    unsigned long long m = __ballot(need);
    if (m) {
      int leader = __ffsll((long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(A.counter, (uint32_t)__popcll(m));
      base = __shfl(base, leader);
      if (need) {
        uint32_t item = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (item >= A.items) {
          mode = M_DONE;
        } else {
          uint32_t slot = item / (uint32_t)A.items_per_pixel, chunk = item % (uint32_t)A.items_per_pixel;
          uint32_t tile = slot >> 6, w = slot & 63u;
          int32_t px = (int32_t)((tile % (uint32_t)A.tiles_x) * 8 + (w & 7u));
          int32_t py = (int32_t)((tile / (uint32_t)A.tiles_x) * 8 + (w >> 3));
          if (px < A.fr.w && py < A.fr.h) {
            pix = (uint32_t)(py * A.fr.w + px);
            s = A.sample_offset + (int32_t)chunk * A.per_item;
            s_end = min(s + A.per_item, A.sample_offset + A.spp);
            acc = make_float3(0, 0, 0);
            mode = M_START;
          }
        }
      }
    }
    if (__ballot(mode != M_DONE) == 0) break;

    bool finish = false;
    // ---- new sample: camera ray, entry into the grid, point location
    if (mode == M_START) {
      int32_t px = (int32_t)(pix % (uint32_t)A.fr.w), py = (int32_t)(pix / (uint32_t)A.fr.w);
      float u0 = uniform01(A.seed, pix, (uint32_t)s, 0, kStreamCamera, 0);
      float u1 = uniform01(A.seed, pix, (uint32_t)s, 0, kStreamCamera, 1);
      float sx = ((2.0f * (((float)px + u0) / (float)A.fr.w)) - 1.0f) * A.fr.tan_x;
      float sy = (1.0f - 2.0f * (((float)py + u1) / (float)A.fr.h)) * A.fr.tan_y;
      o = make_float3(A.fr.pos[0], A.fr.pos[1], A.fr.pos[2]);
      d = normalize3(make_float3((A.fr.f[0] + sx * A.fr.r[0]) + sy * A.fr.u[0],
                                 (A.fr.f[1] + sx * A.fr.r[1]) + sy * A.fr.u[1],
                                 (A.fr.f[2] + sx * A.fr.r[2]) + sy * A.fr.u[2]));
      float3 p;
      int64_t c = -1;
      if (enter_cube(o, d, p)) c = med.locate(p);
      if (c < 0) {
        L = make_float3(A.env[0], A.env[1], A.env[2]);
        finish = true;
      } else {
        cell = (uint32_t)c;
        o = p;
        t = 0.0f;
        beta = make_float3(1.0f, 1.0f, 1.0f);
        L = make_float3(0, 0, 0);
        bounce = 0;
        jf = 0;
        jn = 0;
        steps = 0;
        tau = exp_tau(uniform01(A.seed, pix, (uint32_t)s, 0, kStreamFlight, jf++));
        mode = M_TRACK;
      }
    }
    // ---- one walk step (main path or light ray)
    if (mode == M_TRACK || mode == M_SHADOW) {
      bool shadow_done = false;
      if (steps >= A.max_steps) {
        c_trunc++;
        finish = true;
      } else {
        Step st = med.step(cell, o, d, t);
        steps++;
        c_steps++;
        if (mode == M_TRACK) {
          if (!st.ok) {
            L.x = L.x + beta.x * A.env[0];
            L.y = L.y + beta.y * A.env[1];
            L.z = L.z + beta.z * A.env[2];
            c_esc++;
            finish = true;
          } else {
            float sg = st.sigma, sb = st.majorant;
            bool collided = false;
            float tc = 0.0f;
            if (sb > 0.0f) {
              float dtau = sb * (st.te - t);
              while (tau < dtau) {
                tc = t + tau / sb;
                bool real = true;
                if (sg < sb) real = uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamFlight, jf++) < sg / sb;
                if (real) {
                  collided = true;
                  break;
                }
                c_null++;
                t = tc;
                tau = exp_tau(uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamFlight, jf++));
                dtau = sb * (st.te - t);
              }
              if (!collided) tau = tau - dtau;
            }
            if (collided) {
              c_real++;
              float3 x = make_float3(o.x + tc * d.x, o.y + tc * d.y, o.z + tc * d.z);
              bounce++;
              jf = 0;
              jn = 0;
              beta.x = beta.x * A.albedo;
              beta.y = beta.y * A.albedo;
              beta.z = beta.z * A.albedo;
              dsave = d;
              o = x;
              d = sun;
              t = 0.0f;
              cell_x = cell;
              od = 0.0f;
              tr = 1.0f;
              if (A.transmittance != 0) tau = exp_tau(uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamLight, jn++));
              mode = M_SHADOW;
            } else {
              t = st.te;
              if (st.next < 0) {
                L.x = L.x + beta.x * A.env[0];
                L.y = L.y + beta.y * A.env[1];
                L.z = L.z + beta.z * A.env[2];
                c_esc++;
                finish = true;
              } else {
                cell = (uint32_t)st.next;
              }
            }
          }
        } else {  // light ray
          if (!st.ok) {
            shadow_done = true;
          } else {
            float sg = st.sigma, sb = st.majorant;
            if (A.transmittance == 0) {
              od = od + sg * (st.te - t);
            } else if (sb > 0.0f) {
              float dtau = sb * (st.te - t);
              while (tau < dtau) {
                t = t + tau / sb;
                if (A.transmittance == 1) {
                  tr = tr * (1.0f - sg / sb);
                } else {
                  bool real = true;
                  if (sg < sb) real = uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamLight, jn++) < sg / sb;
                  if (real) {
                    tr = 0.0f;
                    shadow_done = true;
                    break;
                  }
                }
                tau = exp_tau(uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamLight, jn++));
                dtau = sb * (st.te - t);
              }
              if (!shadow_done) tau = tau - dtau;
            }
            if (A.transmittance == 1 && tr == 0.0f) shadow_done = true;
            if (!shadow_done) {
              t = st.te;
              if (st.next < 0) shadow_done = true;
              else cell = (uint32_t)st.next;
            }
          }
        }
      }
      if (shadow_done) {
        float Tr = A.transmittance == 0 ? (float)exp(-(double)od) : tr;
        float mu = (dsave.x * sun.x + dsave.y * sun.y) + dsave.z * sun.z;
        float ph = hg_pdf(A.g, mu);
        L.x = L.x + ((beta.x * ph) * A.E[0]) * Tr;
        L.y = L.y + ((beta.y * ph) * A.E[1]) * Tr;
        L.z = L.z + ((beta.z * ph) * A.E[2]) * Tr;
        if ((int32_t)bounce >= A.max_bounces) {
          finish = true;
        } else {
          float v1 = uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamPhase, 0);
          float v2 = uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamPhase, 1);
          d = hg_scatter(dsave, A.g, v1, v2);
          t = 0.0f;
          cell = cell_x;
          tau = exp_tau(uniform01(A.seed, pix, (uint32_t)s, bounce, kStreamFlight, jf++));
          mode = M_TRACK;
        }
      }
    }
    // ---- sample finished: accumulate, next sample or next work item
    if (finish) {
      acc.x = acc.x + L.x;
      acc.y = acc.y + L.y;
      acc.z = acc.z + L.z;
      s++;
      if (s < s_end) {
        mode = M_START;
      } else {
        float* px = A.out + 3 * (size_t)pix;
        if (A.accumulate) {
          atomicAdd(px, acc.x);
          atomicAdd(px + 1, acc.y);
          atomicAdd(px + 2, acc.z);
        } else {
          px[0] = acc.x / (float)A.spp;
          px[1] = acc.y / (float)A.spp;
          px[2] = acc.z / (float)A.spp;
        }
        mode = M_FETCH;
      }
    }
  }
  // ---- counters: wave reduction, one atomic per wave and counter
  unsigned long long v[5] = {c_steps, c_null, c_real, c_esc, c_trunc};
#pragma unroll
  for (int q = 0; q < 5; q++) {
    unsigned long long x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0 && x) atomicAdd(A.stats + q, x);
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_zero_f32(float* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

__global__ void k_scale_f32(float* p, int64_t n, float div) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = p[i] / div;
}

__global__ void k_locate(TetMedium med, const float* __restrict__ pts, int64_t count, int64_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float3 p = make_float3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
  bool in = p.x >= 0.0f && p.x <= 1.0f && p.y >= 0.0f && p.y <= 1.0f && p.z >= 0.0f && p.z <= 1.0f;
  out[i] = in ? med.locate(p) : -1;
}

// ---------------------------------------------------------------- host
static int render_common(int kind, const tet_grid* g, const tet_density* dens, const tet_camera* cam,
                         const tet_medium* medm, const tet_light* light, int32_t spp, uint64_t seed,
                         const tet_render_opts* opts_in, float* out_rgb, int32_t on_device, hipStream_t st,
                         tet_render_stats* stats) {
  if (int rc = check_camera(cam)) return rc;
  if (!medm || !light || !out_rgb) return fail(TET_ERR_INVALID_ARG, "render: NULL medium, light or output");
  if (spp < 1) return fail(TET_ERR_INVALID_ARG, "render: spp must be >= 1");
  if (!(medm->g > -1.0f && medm->g < 1.0f) || !(medm->albedo >= 0.0f))
    return fail(TET_ERR_INVALID_ARG, "render: medium needs albedo >= 0 and -1 < g < 1");
  tet_render_opts o;
  if (opts_in) o = *opts_in;
  else tet_render_opts_defaults(&o);
  if (o.max_bounces < 1 || o.transmittance < 0 || o.transmittance > 2 || o.max_steps_per_path < 1 ||
      o.sample_offset < 0 || o.samples_per_item < 0 || o.block_size < 0 || o.block_size > 1024 ||
      (o.block_size % 64) != 0 || o.blocks_per_cu < 0)
    return fail(TET_ERR_INVALID_ARG, "render: bad options");
  int64_t npix = (int64_t)cam->width * cam->height;
  int per_item = (o.samples_per_item <= 0 || o.samples_per_item > spp) ? spp : o.samples_per_item;
  int ipp = (spp + per_item - 1) / per_item;
  int tiles_x = (cam->width + 7) / 8, tiles_y = (cam->height + 7) / 8;
  int64_t items = (int64_t)tiles_x * tiles_y * 64 * ipp;
  if (items >= (1ll << 32) || npix > (1ll << 31) - 1)
    return fail(TET_ERR_INVALID_ARG, "render: image too large");

  RenderArgs A;
  memset(&A, 0, sizeof(A));
  make_frame(*cam, &A.fr);
  A.albedo = medm->albedo;
  A.g = medm->g;
  for (int i = 0; i < 3; i++) {
    A.sun[i] = light->sun_dir[i];
    A.E[i] = light->sun_irradiance[i];
    A.env[i] = light->env_radiance[i];
  }
  A.spp = spp;
  A.sample_offset = o.sample_offset;
  A.per_item = per_item;
  A.items_per_pixel = ipp;
  A.max_bounces = o.max_bounces;
  A.transmittance = o.transmittance;
  A.max_steps = o.max_steps_per_path;
  A.seed = seed;
  A.items = (uint32_t)items;
  A.tiles_x = tiles_x;
  A.accumulate = ipp > 1;

  // scratch: counter + 5 stats + image when the output is on the host
  size_t img_bytes = (size_t)npix * 3 * sizeof(float);
  size_t scratch = 64 + (on_device ? 0 : img_bytes);
  char* sc = (char*)dev_alloc(scratch);
  if (!sc) return fail(TET_ERR_OUT_OF_MEMORY, "render: scratch");
  struct Free {
    void* p;
    ~Free() { dev_free(p); }
  } fr_{sc};
  A.counter = (uint32_t*)sc;
  A.stats = (unsigned long long*)(sc + 16);
  A.out = on_device ? out_rgb : (float*)(sc + 64);

  hipDeviceProp_t prop;
  int dev = 0;
  TV_HIP(hipGetDevice(&dev));
  TV_HIP(hipGetDeviceProperties(&prop, dev));
  int bs = o.block_size ? o.block_size : 256;
  int bpc = o.blocks_per_cu ? o.blocks_per_cu : 8;
  int64_t grid = (int64_t)prop.multiProcessorCount * bpc;
  int64_t need = (items + bs - 1) / bs;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;

  hipEvent_t e0, e1;
  TV_HIP(hipEventCreate(&e0));
  TV_HIP(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (uint32_t*)sc, 16);
  if (A.accumulate)
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((npix * 3 + 255) / 256)), dim3(256), 0, st, A.out, npix * 3);
  TV_HIP(hipEventRecord(e0, st));
  if (kind == 0) {
    TetMedium m{g->rec, g->keys, g->n, g->max_depth};
    A.rec = g->rec;
    A.keys = g->keys;
    A.n = g->n;
    A.dmax = g->max_depth;
    hipLaunchKernelGGL(k_render<TetMedium>, dim3((unsigned)grid), dim3(bs), 0, st, A, m);
  } else {
    VoxelMedium m{dens->data, dens->n, dens->density_scale};
    hipLaunchKernelGGL(k_render<VoxelMedium>, dim3((unsigned)grid), dim3(bs), 0, st, A, m);
  }
  TV_HIP(hipGetLastError());
  TV_HIP(hipEventRecord(e1, st));
  if (A.accumulate)
    hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)((npix * 3 + 255) / 256)), dim3(256), 0, st, A.out, npix * 3,
                       (float)spp);
  unsigned long long hs[5] = {0, 0, 0, 0, 0};
  TV_HIP(hipMemcpyAsync(hs, A.stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (!on_device) TV_HIP(hipMemcpyAsync(out_rgb, A.out, img_bytes, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  float ms = 0.0f;
  TV_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (stats) {
    stats->tet_steps = (int64_t)hs[0];
    stats->null_collisions = (int64_t)hs[1];
    stats->real_collisions = (int64_t)hs[2];
    stats->escapes = (int64_t)hs[3];
    stats->truncated = (int64_t)hs[4];
    stats->ms = ms;
  }
  return TET_OK;
}

int render_grid(const tet_grid* g, const tet_camera* cam, const tet_medium* m, const tet_light* l, int32_t spp,
                uint64_t seed, const tet_render_opts* o, float* out, int32_t on_device, hipStream_t st,
                tet_render_stats* stats) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_render: grid is NULL");
  return render_common(0, g, nullptr, cam, m, l, spp, seed, o, out, on_device, st, stats);
}

int render_voxels(const tet_density* dens, const tet_camera* cam, const tet_medium* m, const tet_light* l,
                  int32_t spp, uint64_t seed, const tet_render_opts* o, float* out, int32_t on_device,
                  hipStream_t st, tet_render_stats* stats) {
  if (!dens || !dens->data) return fail(TET_ERR_INVALID_ARG, "dda_render: density is NULL");
  int32_t n = dens->n;
  if (n < 1 || n > 1024 || (n & (n - 1))) return fail(TET_ERR_INVALID_ARG, "dda_render: n must be a power of two <= 1024");
  if (dens->on_device) return render_common(1, nullptr, dens, cam, m, l, spp, seed, o, out, on_device, st, stats);
  size_t bytes = (size_t)n * n * n * 4;
  float* dd = (float*)dev_alloc(bytes);
  if (!dd) return fail(TET_ERR_OUT_OF_MEMORY, "dda_render: density copy");
  struct Free {
    void* p;
    ~Free() { dev_free(p); }
  } f_{dd};
  TV_HIP(hipMemcpyAsync(dd, dens->data, bytes, hipMemcpyHostToDevice, st));
  tet_density dv = *dens;
  dv.data = dd;
  dv.on_device = 1;
  return render_common(1, nullptr, &dv, cam, m, l, spp, seed, o, out, on_device, st, stats);
}

int locate_points(const tet_grid* g, const float* pts, int64_t count, int64_t* out, int32_t on_device,
                  hipStream_t st) {
  if (!g || count < 0 || (count && (!pts || !out))) return fail(TET_ERR_INVALID_ARG, "tet_locate: bad arguments");
  if (count == 0) return TET_OK;
  const float* dp = pts;
  int64_t* dout = out;
  char* tmp = nullptr;
  if (!on_device) {
    tmp = (char*)dev_alloc(count * 12 + count * 8 + 16);
    if (!tmp) return fail(TET_ERR_OUT_OF_MEMORY, "tet_locate: scratch");
    dout = (int64_t*)tmp;
    dp = (const float*)(tmp + count * 8);
    TV_HIP(hipMemcpyAsync((void*)dp, pts, count * 12, hipMemcpyHostToDevice, st));
  }
  struct Free {
    void* p;
    ~Free() { if (p) dev_free(p); }
  } f_{tmp};
  TetMedium m{g->rec, g->keys, g->n, g->max_depth};
  hipLaunchKernelGGL(k_locate, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, m, dp, count, dout);
  TV_HIP(hipGetLastError());
  if (!on_device) TV_HIP(hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

}  // namespace tv
