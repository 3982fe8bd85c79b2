// render.hip -- Monte Carlo volumetric path tracing through the tet grid
// (paper, "Volumetric Path Tracing": Algorithm 1 and "Path Tracing within
// Tetrahedral Grids").
//
// Two kernels per pass of samples:
//   k_raygen  -- one thread per (pixel, sample): camera ray, entry into the
//                grid, point location and the first free-flight depth,
//                written as a 32-byte entry record (coherent, no divergence
//                beyond the point-location search);
//   k_render  -- persistent: every lane runs a small state machine over its
//                own paths (fetch work -> load an entry -> walk steps of the
//                main path -> walk steps of the light (shadow) ray ->
//                scatter).  Each loop iteration advances every walking lane
//                by one cell, so lanes whose paths differ in length stay
//                busy; idle lanes take new work items from a device counter
//                with one atomic per wave (ballot + popcount).  All rare
//                events (collision, light estimate and phase sampling,
//                escape, end of sample, new work) sit in one section the
//                wave enters only when some lane needs it; the common
//                iteration is a bare walk step.
//
// One walk step reads one 48-byte tet record (face plane offsets, face
// orientation codes, 4 neighbour links, extinction, majorant) and evaluates
// only faces whose outward normal faces the ray (n.d > 0, at most 3).  The
// dot products of the segment's origin and direction with the 9 possible
// face directions are computed once per segment into a per-lane LDS table,
// so a face costs one LDS read pair and a sign flip; every value is rounded
// exactly as the direct FP32 dot product would be.  The free flight is delta tracking against the
// per-tet majorant with an optical depth carried across cells; real
// collisions scatter by Henyey-Greenstein after a next-event estimate of the
// directional light (transmittance by walking the light ray to the grid
// boundary); paths leaving the grid see the constant environment.
//
// The same kernel, instantiated on the voxel grid (Amanatides-Woo steps),
// is the regular-grid reference renderer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "nrc.h"

namespace tv {

// Entry of one camera sample into the grid (32 bytes): entry point, tet
// (kMiss if the ray misses the grid), direction, first free-flight depth.
struct alignas(16) RayEntry {
  float px, py, pz;
  uint32_t cell;
  float dx, dy, dz;
  float tau;
};
constexpr uint32_t kMiss = 0xFFFFFFFFu;

// One scene of a batch (several grids rendered by one launch sequence).
// Work items and entry records of all scenes are concatenated; a scene's
// items start at a multiple of 64, so the 64-item batches waves take never
// straddle two scenes.
// Extra per-tet data a scene may carry: channels (null = absent) with the
// emitted radiance per unit temperature, and the density model inside the
// tets (0 = constant; 1 linear coefficients; 2 voxel lookup in an n^3
// volume times a scale).
struct ExtArgs {
  const float* ch_t;
  const float* ch_a;
  const float* ch_g;
  float emission[3];
  int32_t model;
  const float4* mcoef;
  const float* mdens;
  int32_t mn;
  float mscale;
};

struct SceneDesc {
  Frame fr;
  float albedo, g;
  float sun[3], E[3], env[3];
  int32_t spp, tiles_x;
  uint64_t seed;
  uint32_t s0;       // first sample index
  uint32_t items;    // slots x spp (the scene's work items, one sample each)
  uint32_t item0;    // first work item (multiple of 64)
  uint32_t pad0;
  uint64_t entry0;   // first entry record
  uint64_t pix0;     // first pixel in the concatenated images
  const void* rec;   // traversal records (TetRec32 or TetRec)
  const uint64_t* keys;
  const uint32_t* kidx;
  int64_t n;
  int32_t dmax, kbits;
  float* out;
  ExtArgs ex;
};

// Largest k < n with key(k) <= v (key ascending, key(0) = 0).
template <class F>
__device__ inline int scene_search(int n, uint64_t v, F key) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (key(mid) <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// A light ray whose walk is deferred: its origin (the real collision), the
// collision's tet, the light estimate's weight per channel (throughput after
// the albedo x phase function x irradiance) and the pixel it adds to.
struct alignas(16) LightRec {
  float x, y, z;
  uint32_t cell;
  float w0, w1, w2;
  uint32_t pix;
};

struct RenderArgs {
  Frame fr;
  float albedo, g;
  float sun[3], E[3], env[3];
  int32_t spp;          // samples per pixel of the whole render (divisor)
  int32_t pass_start;   // first sample index of this pass
  int32_t pass_spp;     // samples of this pass
  int32_t per_item, items_per_pixel, max_bounces, transmittance;
  uint32_t max_steps;
  uint64_t seed;
  uint32_t items, slots;
  uint32_t range_size;  // work items per XCD range (8 contiguous ranges)
  uint32_t batch;       // work items a wave takes per atomic
  int32_t event_wait;   // lanes waiting for an event before the wave handles events
  int32_t tiles_x;
  const RayEntry* entries;
  float* out;
  uint32_t* counter;
  unsigned long long* stats;
  int accumulate;
  // radiance cache
  int32_t train;         // work items are training paths (pixel from train_pixel, sample = item)
  uint32_t npix;         // width * height
  int32_t truncate;      // real vertex where a path queries the cache
  int32_t rec_vertices;  // vertices recorded per training path
  float4* qbuf;          // cache queries of the pass, compacted: (x, sigma), (d, beta)
  uint32_t* qpix;        // their pixels
  uint32_t* qcount;      // queries so far (one atomic per wave)
  float4* vrec;          // training-path vertex records
  float4* path_l;        // training-path radiance and vertex count
  const tet_nrc* nrc;    // host handle (the query pass), never read on the device
  uint32_t train_items;  // cache mode 1: the first items are training paths (first pass only)
  uint32_t train_ent0;   // their entry records follow the image's
  uint64_t train_seed;   // their Philox key
  // batch of scenes
  const SceneDesc* scenes;
  int32_t nscenes;
  uint64_t total_entries;
  ExtArgs ex;  // channels and density model of a single-scene render
  // deferred light rays (defer != 0): block b of the tracing kernel queues
  // its light rays at lq + b * lq_region (lq_count[b] of them), walked after
  // the pass in the order of their start tets
  LightRec* lq;
  uint32_t* lq_count;
  uint32_t lq_cap;
  uint32_t lq_region;
  int32_t defer;
};

// Extinction at o + t d inside tet `cell` under the grid's density model:
// linear ((c0 + gx x) + gy y) + gz z, or the scale times the voxel
// floor(x n) (indices clamped); FP32.
__device__ inline float model_sigma(const ExtArgs& X, uint32_t cell, float3 o, float3 d, float t) {
  const float x0 = o.x + t * d.x, x1 = o.y + t * d.y, x2 = o.z + t * d.z;
  if (X.model == 1) {
    const float4 c = X.mcoef[cell];
    return ((c.x + c.y * x0) + c.z * x1) + c.w * x2;
  }
  const int32_t n = X.mn;
  const float fn = (float)n;
  int64_t i = (int64_t)floorf(x0 * fn), j = (int64_t)floorf(x1 * fn), k = (int64_t)floorf(x2 * fn);
  i = i < 0 ? 0 : (i >= n ? n - 1 : i);
  j = j < 0 ? 0 : (j >= n ? n - 1 : j);
  k = k < 0 ? 0 : (k >= n ? n - 1 : k);
  return X.mscale * X.mdens[i + (int64_t)n * (j + (int64_t)n * k)];
}

// Pixel of training path j: floor(w npix / 2^24), w = the upper 24 bits of
// word 0 of Philox(counter (j, 0, 4, 0)).
__device__ inline uint32_t train_pixel(uint64_t seed, uint32_t j, uint32_t npix) {
  uint4 r = philox10(make_uint4(j, 0u, 4u, 0u), (uint32_t)seed, (uint32_t)(seed >> 32));
  return (uint32_t)(((uint64_t)(r.x >> 8) * npix) >> 24);
}

// pixel of a slot: 8x8 tiles in row-major tile order
__device__ inline bool slot_pixel(uint32_t slot, int32_t tiles_x, int32_t w, int32_t h, int32_t& px, int32_t& py) {
  uint32_t tile = slot >> 6, q = slot & 63u;
  px = (int32_t)((tile % (uint32_t)tiles_x) * 8 + (q & 7u));
  py = (int32_t)((tile / (uint32_t)tiles_x) * 8 + (q >> 3));
  return px < w && py < h;
}

struct Step {
  float te, sigma, majorant;
  int32_t next;  // -1: leaves the grid
  bool ok;       // false: no exit face
};

// ---------------------------------------------------------------- tet medium
template <int K>
__device__ inline void descend_point(int32_t v[4][3], uint64_t& h, uint32_t& cls, const uint32_t* __restrict__ shapes,
                                     const double P[3]) {
  const uint32_t w = shapes[cls];
  int32_t z[3], u[3];
  shape_bisector<K>(v, w, z, u);
  double side = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const double t = P[i] - (double)z[i];
    if (u[i]) side = side + (u[i] > 0 ? t : -t);
  }
  cls = side >= 0.0 ? (w >> 8) & 255u : (w >> 16) & 255u;
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
__device__ inline int64_t locate_point(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ kidx, int kbits,
                                       int dmax, const uint32_t* __restrict__ shapes, float3 p) {
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
  uint32_t cls = shapes[kShapeWords + r];
  for (int d = 0; d < dmax; d += 3) {
    descend_point<3>(v, h, cls, shapes, P);
    if (d + 1 < dmax) descend_point<2>(v, h, cls, shapes, P);
    if (d + 2 < dmax) descend_point<1>(v, h, cls, shapes, P);
  }
  return search_keys_idx(keys, kidx, kbits, h << (60 - dmax));
}

struct TetMedium {
  static constexpr float kOriginScale = 1.0f;
  const TetRec* __restrict__ rec;
  const uint64_t* __restrict__ keys;
  int64_t n;
  int dmax;
  const uint32_t* __restrict__ shapes;
  const uint32_t* __restrict__ kidx;
  int kbits;
  __device__ inline int64_t locate(float3 p) const { return locate_point(keys, kidx, kbits, dmax, shapes, p); }
  __device__ inline float sigma_at(uint32_t cell) const { return rec[cell].sigma; }
  // Exit of the tet along the segment whose direction-dot table is `tab`
  // (tab[N] = dir_N . d, tab[9 + N] = dir_N . o) from t: faces with
  // n.d > 0 are candidates; the exit face has the smallest exact quotient
  // num / den (exact FP64 cross products, lowest face on ties); one FP32
  // division gives the exit distance.  Branchless, so the whole record is
  // loaded at once.
  __device__ inline Step step(uint32_t cell, float3, float3, const float* tab, float t) const {
    const float4* q = (const float4*)(rec + cell);
    const float4 r0 = q[0], r1 = q[1], r2 = q[2];
    const uint32_t codes = __float_as_uint(r2.x);
    const float off[4] = {r0.x, r0.y, r0.z, r0.w};
    const uint32_t link[4] = {__float_as_uint(r1.x), __float_as_uint(r1.y), __float_as_uint(r1.z),
                              __float_as_uint(r1.w)};
    bool any = false;
    float bnum = 0.0f, bden = 1.0f;
    uint32_t blink = kBoundary;
    // the four faces' table entries, all read before any is used
    float tden[4], tdot[4];
#pragma unroll
    for (int f = 0; f < 4; f++) {
      const uint32_t c = (codes >> (8 * f)) & 0xFFu;
      tden[f] = tab[c >> 1];
      tdot[f] = tab[9 + (c >> 1)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int f = 0; f < 4; f++) {
      uint32_t c = (codes >> (8 * f)) & 0xFFu;
      uint32_t sg = c << 31;
      float den = __uint_as_float(__float_as_uint(tden[f]) ^ sg);
      float dot = __uint_as_float(__float_as_uint(tdot[f]) ^ sg);
      float num = off[f] - dot;
      bool cand = den > 0.0f;
      bool better = cand && (!any || (double)num * (double)bden < (double)bnum * (double)den);
      bnum = better ? num : bnum;
      bden = better ? den : bden;
      blink = better ? link[f] : blink;
      any = any || cand;
    }
    Step s;
    float bt = bnum / bden;
    s.sigma = r2.y;
    s.majorant = r2.z;
    s.ok = any;
    s.te = bt > t ? bt : t;
    s.next = (!any || blink == kBoundary) ? -1 : (int32_t)(blink >> 2);
    return s;
  }
};

// Same walk on the compact 32-byte records (bitwise the same values).  The
// LDS table holds origin dots scaled by 2^20 (exact), so the integer
// offsets need no scaling: num * 2^20 = offset - dot * 2^20 exactly, the
// quotient comparisons are scale-free, and one final multiply by 2^-20
// (exact) gives the exit distance.  The running best starts at the
// quotient 1/0 = +inf, which every candidate beats.
struct TetMedium32 {
  static constexpr float kOriginScale = 0x1p20f;  // origin dots stored times 2^20
  const TetRec32* __restrict__ rec;
  const uint64_t* __restrict__ keys;
  int64_t n;
  int dmax;
  const uint32_t* __restrict__ shapes;
  const uint32_t* __restrict__ kidx;
  int kbits;
  __device__ inline int64_t locate(float3 p) const { return locate_point(keys, kidx, kbits, dmax, shapes, p); }
  __device__ inline float sigma_at(uint32_t cell) const { return __uint_as_float(rec[cell].w[3]); }
  __device__ inline Step step(uint32_t cell, float3, float3, const float* tab, float t) const {
    // byte offset in 32 bits (cell < 2^27): a uniform base takes the load's
    // scalar-base form
    const uint4* q = (const uint4*)((const char*)rec + (cell << 5));
    const uint4 a = q[0], b = q[1];
    uint32_t o1 = (uint32_t)((((uint64_t)a.y << 32) | a.x) >> 23);
    uint32_t o2 = (uint32_t)((((uint64_t)a.z << 32) | a.y) >> 14);
    const int32_t ioff[4] = {((int32_t)(a.x << 9)) >> 9, ((int32_t)(o1 << 9)) >> 9, ((int32_t)(o2 << 9)) >> 9,
                             ((int32_t)(a.z << 4)) >> 9};
    const uint32_t lw[4] = {b.x, b.y, b.z, b.w};
    // the four faces' table entries, all read before any is used
    float tden[4], tdot[4];
#pragma unroll
    for (int f = 0; f < 4; f++) {
      // direction index N (bits 27..30) as one bit-field extract: left to
      // the compiler it becomes shift, mask and add before the address add
      uint32_t dn;
      asm("v_bfe_u32 %0, %1, 27, 4" : "=v"(dn) : "v"(lw[f]));
      const float* e = tab + dn;
      tden[f] = e[0];
      tdot[f] = e[9];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the four reads ahead of their uses
    float bnum, bden;
    uint32_t bw;  // link word of the best face (all ones: none yet)
    {  // face 0 against the start quotient 1/0: it wins exactly when it is a candidate
      uint32_t sg = lw[0] & 0x80000000u;
      float den = __uint_as_float(__float_as_uint(tden[0]) ^ sg);
      float dot = __uint_as_float(__float_as_uint(tdot[0]) ^ sg);
      float num = (float)ioff[0] - dot;
      const bool cand = den > 0.0f;
      bnum = cand ? num : 1.0f;
      // -0 when there is no candidate: the same comparisons as +0 below (a
      // candidate's 1 * den is > 0), and a plain select rather than a max
      bden = cand ? den : -0.0f;
      bw = cand ? lw[0] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int f = 1; f < 4; f++) {
      uint32_t sg = lw[f] & 0x80000000u;
      float den = __uint_as_float(__float_as_uint(tden[f]) ^ sg);
      float dot = __uint_as_float(__float_as_uint(tdot[f]) ^ sg);
      float num = (float)ioff[f] - dot;
      bool better = den > 0.0f && (double)num * (double)bden < (double)bnum * (double)den;
      bnum = better ? num : bnum;
      bden = better ? den : bden;
      bw = better ? lw[f] : bw;
    }
    const uint32_t blink = bw & kLink27Boundary;
    Step s;
    bool any = bden > 0.0f;
    float bt = (bnum / bden) * 0x1p-20f;
    s.sigma = __uint_as_float(a.w);
    s.majorant = s.sigma;
    s.ok = any;
    s.te = bt > t ? bt : t;
    s.next = (!any || blink == kLink27Boundary) ? -1 : (int32_t)blink;
    return s;
  }
};

// ---------------------------------------------------------------- voxel medium
struct VoxelMedium {
  static constexpr float kOriginScale = 1.0f;
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
  __device__ inline float sigma_at(uint32_t cell) const { return scale * dens[cell]; }
  __device__ inline Step step(uint32_t cell, float3 o, float3 d, const float*, float t) const {
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

// ---------------------------------------------------------------- kernels
// Camera ray of sample s of pixel (px, py), its entry into the grid, the
// entry tet and the first free-flight depth.
template <class Med>
__device__ inline RayEntry camera_entry(const Frame& fr, uint64_t seed, const Med& med, int32_t px, int32_t py,
                                        uint32_t pix, uint32_t s) {
  uint2 u = uniform01x2(seed, pix, s, 0, kStreamCamera, 0);
  float u0 = u01(u.x), u1 = u01(u.y);
  float sx = ((2.0f * (((float)px + u0) / (float)fr.w)) - 1.0f) * fr.tan_x;
  float sy = (1.0f - 2.0f * (((float)py + u1) / (float)fr.h)) * fr.tan_y;
  float3 o = make_float3(fr.pos[0], fr.pos[1], fr.pos[2]);
  float3 d = normalize3(make_float3((fr.f[0] + sx * fr.r[0]) + sy * fr.u[0], (fr.f[1] + sx * fr.r[1]) + sy * fr.u[1],
                                    (fr.f[2] + sx * fr.r[2]) + sy * fr.u[2]));
  float3 p = o;
  int64_t c = -1;
  if (enter_cube(o, d, p)) c = med.locate(p);
  RayEntry r;
  r.px = p.x;
  r.py = p.y;
  r.pz = p.z;
  r.cell = c < 0 ? kMiss : (uint32_t)c;
  r.dx = d.x;
  r.dy = d.y;
  r.dz = d.z;
  r.tau = c < 0 ? 0.0f : exp_tau(uniform01(seed, pix, s, 0, kStreamFlight, 0));
  return r;
}

__device__ inline RayEntry miss_entry() {
  RayEntry z;
  memset(&z, 0, sizeof(z));
  z.cell = kMiss;
  return z;
}

// Entry records of every (pixel, sample) of a batch of scenes.
template <class Med>
__global__ __launch_bounds__(256) void k_raygen_batch(RenderArgs A, Med med, RayEntry* __restrict__ entries) {
  uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A.total_entries) return;
  const int k = scene_search(A.nscenes, e, [&](int i) { return A.scenes[i].entry0; });
  const SceneDesc& S = A.scenes[k];
  uint64_t local = e - S.entry0;
  uint32_t slot = (uint32_t)(local / (uint32_t)S.spp);
  uint32_t s = S.s0 + (uint32_t)(local % (uint32_t)S.spp);
  int32_t px, py;
  if (!slot_pixel(slot, S.tiles_x, S.fr.w, S.fr.h, px, py)) {
    entries[e] = miss_entry();
    return;
  }
  Med m = med;
  m.rec = (decltype(m.rec))S.rec;
  m.keys = S.keys;
  m.kidx = S.kidx;
  m.kbits = S.kbits;
  m.n = S.n;
  m.dmax = S.dmax;
  entries[e] = camera_entry(S.fr, S.seed, m, px, py, (uint32_t)(py * S.fr.w + px), s);
}

// Zeroes (zero != 0) or divides by spp every pixel of a batch's images.
__global__ void k_batch_images(const SceneDesc* __restrict__ sc, int32_t n, uint64_t total_px, int zero) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total_px) return;
  const int k = scene_search(n, i, [&](int j) { return sc[j].pix0; });
  float* o = sc[k].out + 3 * (i - sc[k].pix0);
  if (zero) {
    o[0] = 0.0f;
    o[1] = 0.0f;
    o[2] = 0.0f;
  } else {
    float div = (float)sc[k].spp;
    o[0] = o[0] / div;
    o[1] = o[1] / div;
    o[2] = o[2] / div;
  }
}

template <class Med>
__global__ __launch_bounds__(256) void k_raygen(RenderArgs A, Med med, RayEntry* __restrict__ entries) {
  uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (uint64_t)A.slots * (uint64_t)A.pass_spp) return;
  uint32_t pix, s;
  int32_t px, py;
  if (A.train) {
    s = (uint32_t)e;
    pix = train_pixel(A.seed, s, A.npix);
    px = (int32_t)(pix % (uint32_t)A.fr.w);
    py = (int32_t)(pix / (uint32_t)A.fr.w);
  } else {
    uint32_t slot = (uint32_t)(e / (uint32_t)A.pass_spp);
    s = (uint32_t)(A.pass_start + (int32_t)(e % (uint32_t)A.pass_spp));
    if (!slot_pixel(slot, A.tiles_x, A.fr.w, A.fr.h, px, py)) {
      entries[e] = miss_entry();  // padding slot of an edge tile: never traced, never queried
      return;
    }
    pix = (uint32_t)(py * A.fr.w + px);
  }
  entries[e] = camera_entry(A.fr, A.seed, med, px, py, pix, s);
}

enum { M_TRACK = 0, M_SHADOW = 1, M_COLLIDE = 2, M_SCATTER = 3, M_ESCAPE = 4, M_FINISH = 5, M_FETCH = 6,
       M_START = 7, M_DONE = 8 };

constexpr int kTabStride = 19;  // floats per lane in the LDS dot table (odd: no bank conflicts)

// Dot products of the 9 face directions with the segment's direction d and
// origin o, each rounded as (n.x a.x + n.y a.y) + n.z a.z would be (its
// zero terms are exact).
__device__ inline void set_segment(float* tab, float3 o, float3 d, float oscale) {
  o = make_float3(o.x * oscale, o.y * oscale, o.z * oscale);
  tab[0] = d.x;
  tab[1] = d.y;
  tab[2] = d.z;
  tab[3] = d.x + d.y;
  tab[4] = d.x - d.y;
  tab[5] = d.x + d.z;
  tab[6] = d.x - d.z;
  tab[7] = d.y + d.z;
  tab[8] = d.y - d.z;
  tab[9] = o.x;
  tab[10] = o.y;
  tab[11] = o.z;
  tab[12] = o.x + o.y;
  tab[13] = o.x - o.y;
  tab[14] = o.x + o.z;
  tab[15] = o.x - o.z;
  tab[16] = o.y + o.z;
  tab[17] = o.y - o.z;
}

// W: occupancy target in waves per SIMD (the register budget follows).
// NRC: 0 plain estimator; 1 paths stop at real vertex A.truncate and leave
// a query for the radiance cache in their entry record; 2 training paths
// (A.train), whose first vertices and final radiance are recorded.
// BATCH: the lanes' samples come from a batch of scenes (A.scenes); each
// lane keeps its sample's scene index and that grid's record pointer, and
// reads the scene's light, medium, seed and image from the table at events.
// EXT: the variant that reads the extra channels and the density model
// (the plain variant carries none of that code).
template <class Med, int W, int NRC, bool BATCH = false, bool EXT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8))) void k_render(RenderArgs A, Med med) {
  __shared__ float s_tab[256 * kTabStride];
  __shared__ uint32_t s_lq;  // light rays this block queued
  float* tab = s_tab + threadIdx.x * kTabStride;
  const int lane = __lane_id();
  int mode = M_FETCH;
  uint32_t pix = 0, ent = 0;  // ent: the sample's entry record
  int32_t s = 0, s_end = 0;
  float3 o = make_float3(0, 0, 0), d = o, dsave = o, L = o, acc = o;
  float beta = 1.0f, t = 0.0f, tau = 0.0f, od = 0.0f;
  uint32_t cell = 0, cell_x = 0, bounce = 0, jf = 0, jn = 0, steps = 0;
  uint32_t n_steps = 0, n_null = 0, n_real = 0, n_esc = 0, n_trunc = 0, n_query = 0;
  int range = blockIdx.x & 7, tried = 0;  // wave-uniform work range state
  uint32_t bnext = 0, bend = 0;          // wave-uniform batch of work items
  const float3 sun0 = make_float3(A.sun[0], A.sun[1], A.sun[2]);
  uint32_t sc = 0, bsc = 0;  // lane's scene; wave-uniform scene of the current batch
  bool trainp = false;       // cache mode 1: the lane's path is a training path
  Med lm = med;              // the lane's medium (its scene's records)
  // plain single-scene walks on tet grids may queue their light rays
  constexpr bool DEFER = NRC != 2 && !BATCH && !std::is_same<Med, VoxelMedium>::value;
  if constexpr (DEFER) {
    if (threadIdx.x == 0) s_lq = 0;
    __syncthreads();
  }
#define TV_SC A.scenes[sc]
#define TV_SEED (BATCH ? TV_SC.seed : ((NRC == 1 && trainp) ? A.train_seed : A.seed))
#define TV_ALBEDO (BATCH ? TV_SC.albedo : A.albedo)
#define TV_G (BATCH ? TV_SC.g : A.g)
#define TV_E(i) (BATCH ? TV_SC.E[i] : A.E[i])
#define TV_ENV(i) (BATCH ? TV_SC.env[i] : A.env[i])
#define TV_OUT (BATCH ? TV_SC.out : A.out)
#define TV_SUN (BATCH ? make_float3(TV_SC.sun[0], TV_SC.sun[1], TV_SC.sun[2]) : sun0)
#define TV_EX (BATCH ? TV_SC.ex : A.ex)

  // real collision at t: start the light ray (right after the walk step, or
  // from the event section for the collisions where a path hands over to the
  // radiance cache)
  // extinction at the collision o + t d, the cache's input there: the
  // tet's, or the density model's at the point
  auto vertex_sigma = [&]() -> float {
    if constexpr (EXT)
      if (TV_EX.model) return model_sigma(TV_EX, cell, o, d, t);
    return lm.sigma_at(cell);
  };
  auto start_light = [&]() {
    n_real++;
    float3 x = make_float3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
    bounce++;
    if ((NRC == 2 || (NRC == 1 && trainp)) && (int32_t)bounce <= A.rec_vertices) {
      uint32_t j = NRC == 2 ? ent : ent - A.train_ent0;
      float4* q = A.vrec + ((size_t)j * (uint32_t)A.rec_vertices + (bounce - 1)) * 3;
      q[0] = make_float4(x.x, x.y, x.z, vertex_sigma());
      q[1] = make_float4(d.x, d.y, d.z, beta);
      q[2] = make_float4(L.x, L.y, L.z, 0.0f);
    }
    jf = 0;
    jn = 0;
    // extra channels of the collision's tet: the emitted radiance by
    // the collision estimator (absorbed part of the collision), then the
    // tet's albedo in place of the medium's
    float alb = TV_ALBEDO;
    if (EXT && TV_EX.ch_a) alb = TV_EX.ch_a[cell];
    if (EXT && TV_EX.ch_t) {
      const float e = (1.0f - alb) * TV_EX.ch_t[cell];
      L.x = L.x + beta * (e * TV_EX.emission[0]);
      L.y = L.y + beta * (e * TV_EX.emission[1]);
      L.z = L.z + beta * (e * TV_EX.emission[2]);
    }
    beta = beta * alb;
    if constexpr (DEFER) {
      // queue the light ray (weight now, walk later); the path goes on to its
      // scatter (training paths of the cache keep their own walks: their
      // records need the light gathered before each vertex)
      if (A.defer && !(NRC == 1 && trainp)) {
        const unsigned long long act = __ballot(1);
        const int lead = __builtin_ctzll(act);
        uint32_t base = 0;
        if (lane == lead) base = atomicAdd(&s_lq, (uint32_t)__popcll(act));  // the block's own count, in LDS
        base = __shfl(base, lead);
        const uint32_t q = base + (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
        if (q < A.lq_region) {  // a full region leaves the walk to the lane
          const float gg = (EXT && TV_EX.ch_g) ? TV_EX.ch_g[cell] : TV_G;
          const float mu = (d.x * sun0.x + d.y * sun0.y) + d.z * sun0.z;
          const float bp = beta * hg_pdf(gg, mu);
          LightRec r;
          r.x = x.x;
          r.y = x.y;
          r.z = x.z;
          r.cell = cell;
          r.w0 = bp * A.E[0];
          r.w1 = bp * A.E[1];
          r.w2 = bp * A.E[2];
          r.pix = pix;
          A.lq[(size_t)blockIdx.x * A.lq_region + q] = r;
          dsave = d;
          o = x;
          t = 0.0f;
          cell_x = cell;
          od = -1.0f;  // no light term at the scatter
          mode = M_SCATTER;
          return;
        }
      }
    }
    dsave = d;
    o = x;
    d = TV_SUN;
    t = 0.0f;
    cell_x = cell;
    od = A.transmittance == 0 ? 0.0f : 1.0f;
    if (A.transmittance != 0) tau = exp_tau(uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamLight, jn++));
    set_segment(tab, o, d, Med::kOriginScale);
    mode = M_SHADOW;
  };

  for (;;) {
    // ================= events: run when enough lanes wait for one, or when
    // no lane is walking (waiting lanes idle meanwhile)
    unsigned long long waiting = __ballot(mode > M_SHADOW);
    if (waiting && (__popcll(waiting) >= A.event_wait || __popcll(waiting) == 64 ||
                    __ballot(mode <= M_SHADOW) == 0)) {
      if (NRC == 1) {  // the cache stands for the rest of the path: append a query
        const bool isq = mode == M_COLLIDE && !trainp && (int32_t)bounce + 1 == A.truncate;
        const unsigned long long qm = __ballot(isq);
        if (qm) {
          const int lead = __builtin_ctzll(qm);
          uint32_t base = 0;
          if (lane == lead) base = atomicAdd(A.qcount, (uint32_t)__popcll(qm));
          base = __shfl(base, lead);
          if (isq) {
            const uint32_t q = base + (uint32_t)__popcll(qm & ((1ull << lane) - 1ull));
            n_real++;
            bounce++;
            float3 x = make_float3(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
            A.qbuf[2 * (size_t)q] = make_float4(x.x, x.y, x.z, vertex_sigma());
            A.qbuf[2 * (size_t)q + 1] = make_float4(d.x, d.y, d.z, beta);
            A.qpix[q] = pix;
            n_query++;
            mode = M_FINISH;
          }
        }
      }
      if (mode == M_COLLIDE) start_light();
      if (mode == M_SCATTER) {  // light ray done: light estimate, then phase sampling
        const float gg = (EXT && TV_EX.ch_g) ? TV_EX.ch_g[cell_x] : TV_G;  // the collision tet's phase parameter
        if (!DEFER || od >= 0.0f) {  // (od < 0: the light ray was queued)
          float Tr = A.transmittance == 0 ? exp_neg(od) : od;
          float mu = (dsave.x * TV_SUN.x + dsave.y * TV_SUN.y) + dsave.z * TV_SUN.z;
          float ph = hg_pdf(gg, mu);
          L.x = L.x + ((beta * ph) * TV_E(0)) * Tr;
          L.y = L.y + ((beta * ph) * TV_E(1)) * Tr;
          L.z = L.z + ((beta * ph) * TV_E(2)) * Tr;
        }
        if ((int32_t)bounce >= A.max_bounces) {
          mode = M_FINISH;
        } else {
          uint2 v = uniform01x2(TV_SEED, pix, (uint32_t)s, bounce, kStreamPhase, 0);
          d = hg_scatter(dsave, gg, u01(v.x), u01(v.y));
          t = 0.0f;
          cell = cell_x;
          tau = exp_tau(uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamFlight, jf++));
          set_segment(tab, o, d, Med::kOriginScale);
          mode = M_TRACK;
        }
      }
      if (mode == M_ESCAPE) {  // left the grid: the environment
        n_esc++;
        L.x = L.x + beta * TV_ENV(0);
        L.y = L.y + beta * TV_ENV(1);
        L.z = L.z + beta * TV_ENV(2);
        mode = M_FINISH;
      }
      if (mode == M_FINISH) {  // sample done: accumulate; next sample or next item
        acc.x = acc.x + L.x;
        acc.y = acc.y + L.y;
        acc.z = acc.z + L.z;
        n_steps += steps;
        steps = 0;
        if (NRC == 2 || (NRC == 1 && trainp))
          A.path_l[NRC == 2 ? ent : ent - A.train_ent0] = make_float4(L.x, L.y, L.z, __uint_as_float(bounce));
        s++;
        if (s < s_end) {
          ent++;
          mode = M_START;
        } else if (NRC == 2 || (NRC == 1 && trainp)) {
          mode = M_FETCH;
        } else {
          float* px = TV_OUT + 3 * (size_t)pix;
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
      // idle lanes take consecutive work items from the wave's batch; a wave
      // refills its batch with one atomic, first from this block's XCD range
      // (blocks are dealt to the 8 XCDs round-robin, so an XCD's L2 serves
      // one band of the image), then from the others.  Consecutive items are
      // samples of one pixel, so lanes walking side by side share records.
      bool need = mode == M_FETCH;
      unsigned long long m = __ballot(need);
      if (m) {
        if (bnext >= bend && tried < 8) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(A.counter + range, A.batch);
          base = __shfl(base, 0);
          uint32_t r0 = (uint32_t)range * A.range_size;
          uint32_t rend = min(r0 + A.range_size, A.items);
          if (r0 >= rend || base >= rend - r0) {  // range drained: move on
            range = (range + 1) & 7;
            tried++;
          } else {
            bnext = r0 + base;
            bend = min(bnext + A.batch, rend);
            if constexpr (BATCH) bsc = (uint32_t)scene_search(A.nscenes, bnext, [&](int i) { return A.scenes[i].item0; });
          }
        }
        if (bnext < bend) {
          uint32_t item = bnext + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
          if (need && item < bend) {
            if constexpr (BATCH) {
              const SceneDesc& S = A.scenes[bsc];
              uint32_t local = item - S.item0;
              int32_t px, py;
              if (local < S.items &&
                  slot_pixel(local / (uint32_t)S.spp, S.tiles_x, S.fr.w, S.fr.h, px, py)) {
                pix = (uint32_t)(py * S.fr.w + px);
                s = (int32_t)(S.s0 + local % (uint32_t)S.spp);
                s_end = s + 1;
                ent = (uint32_t)(S.entry0 + local);
                sc = bsc;
                lm.rec = (decltype(lm.rec))S.rec;
                acc = make_float3(0, 0, 0);
                mode = M_START;
              } else {
                mode = M_FETCH;  // padding item or slot: take another
              }
            } else if (NRC == 2) {
              pix = train_pixel(TV_SEED, item, A.npix);
              s = (int32_t)item;
              s_end = s + 1;
              ent = item;
              acc = make_float3(0, 0, 0);
              mode = M_START;
            } else if (NRC == 1 && item < A.train_items) {
              pix = train_pixel(A.train_seed, item, A.npix);
              s = (int32_t)item;
              s_end = s + 1;
              ent = A.train_ent0 + item;
              trainp = true;
              acc = make_float3(0, 0, 0);
              mode = M_START;
            } else {
              const uint32_t it = NRC == 1 ? item - A.train_items : item;
              if (NRC == 1) trainp = false;
              uint32_t slot = it / (uint32_t)A.items_per_pixel;
              uint32_t chunk = it % (uint32_t)A.items_per_pixel;
              int32_t px, py;
              if (slot_pixel(slot, A.tiles_x, A.fr.w, A.fr.h, px, py)) {
                pix = (uint32_t)(py * A.fr.w + px);
                s = A.pass_start + (int32_t)chunk * A.per_item;
                s_end = min(s + A.per_item, A.pass_start + A.pass_spp);
                ent = slot * (uint32_t)A.pass_spp + (uint32_t)(s - A.pass_start);
                acc = make_float3(0, 0, 0);
                mode = M_START;
              } else {
                mode = M_FETCH;  // padding slot of an edge tile: take another item
              }
            }
          }
          bnext = min(bnext + (uint32_t)__popcll(m), bend);
        } else if (tried >= 8) {
          if (need) mode = M_DONE;
        }
      }
      if (mode == M_START) {  // new sample: its precomputed entry into the grid
        const float4* q = (const float4*)(A.entries + ent);
        float4 a = q[0], b = q[1];
        uint32_t c = __float_as_uint(a.w);
        steps = 0;
        if (c == kMiss) {
          L = make_float3(TV_ENV(0), TV_ENV(1), TV_ENV(2));
          bounce = 0;
          mode = M_FINISH;
        } else {
          o = make_float3(a.x, a.y, a.z);
          d = make_float3(b.x, b.y, b.z);
          tau = b.w;
          cell = c;
          t = 0.0f;
          beta = 1.0f;
          L = make_float3(0, 0, 0);
          bounce = 0;
          jf = 1;  // flight draw 0 of bounce 0 made the entry's depth
          jn = 0;
          set_segment(tab, o, d, Med::kOriginScale);
          mode = M_TRACK;
        }
      }
      if (__ballot(mode != M_DONE) == 0) break;
    }
    // ================= one walk step of the main path or of the light ray
    if (mode <= M_SHADOW) {
      if (steps >= A.max_steps) {
        n_trunc++;
        mode = M_FINISH;  // truncated path keeps what it has gathered
      } else {
        Step st = lm.step(cell, o, d, tab, t);
        steps++;
        float sg = st.sigma, sb = st.majorant;
        if (mode == M_TRACK) {
          if (!st.ok) {
            mode = M_ESCAPE;
          } else {
            bool collided = false;
            float tc = 0.0f;
            if (sb > 0.0f) {
              float dtau = sb * (st.te - t);
              while (tau < dtau) {
                tc = t + tau / sb;
                if (EXT && TV_EX.model) sg = model_sigma(TV_EX, cell, o, d, tc);  // extinction at the tentative point
                bool real = true;
                if (sg < sb) real = uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamFlight, jf++) < sg / sb;
                if (real) {
                  collided = true;
                  break;
                }
                n_null++;
                t = tc;
                tau = exp_tau(uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamFlight, jf++));
                dtau = sb * (st.te - t);
              }
              if (!collided) tau = tau - dtau;
            }
            if (collided) {
              t = tc;
              mode = M_COLLIDE;
              // the lane walks its light ray next iteration (a path that hands
              // over to the cache at this vertex appends its query in the
              // event section instead: that append is wave-wide)
              if (NRC != 1 || trainp || (int32_t)bounce + 1 != A.truncate) start_light();
            } else {
              t = st.te;
              if (st.next < 0) mode = M_ESCAPE;
              else cell = (uint32_t)st.next;
            }
          }
        } else {  // light ray: od holds the optical depth (analytic) or the transmittance
          bool done = !st.ok;
          if (st.ok) {
            if (A.transmittance == 0 && EXT && TV_EX.model) {
              // linear model: exact integral over the segment (trapezoid)
              od = od + (0.5f * (model_sigma(TV_EX, cell, o, d, t) + model_sigma(TV_EX, cell, o, d, st.te))) * (st.te - t);
            } else if (A.transmittance == 0) {
              od = od + sg * (st.te - t);
            } else if (sb > 0.0f) {
              float dtau = sb * (st.te - t);
              while (tau < dtau) {
                t = t + tau / sb;
                if (EXT && TV_EX.model) sg = model_sigma(TV_EX, cell, o, d, t);
                if (A.transmittance == 1) {
                  od = od * (1.0f - sg / sb);
                } else {
                  bool real = true;
                  if (sg < sb) real = uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamLight, jn++) < sg / sb;
                  if (real) {
                    od = 0.0f;
                    done = true;
                    break;
                  }
                }
                tau = exp_tau(uniform01(TV_SEED, pix, (uint32_t)s, bounce, kStreamLight, jn++));
                dtau = sb * (st.te - t);
              }
              if (!done) tau = tau - dtau;
            }
            if (A.transmittance == 1 && od == 0.0f) done = true;
            if (!done) {
              t = st.te;
              if (st.next < 0) done = true;
              else cell = (uint32_t)st.next;
            }
          }
          if (done) mode = M_SCATTER;
        }
      }
    }
  }
#undef TV_EX
#undef TV_SUN
#undef TV_OUT
#undef TV_ENV
#undef TV_E
#undef TV_G
#undef TV_ALBEDO
#undef TV_SEED
#undef TV_SC
  if constexpr (DEFER) {
    if (A.defer) {
      __syncthreads();
      if (threadIdx.x == 0) A.lq_count[blockIdx.x] = min(s_lq, A.lq_region);
    }
  }
  // ---- counters: wave reductions, one atomic per wave and counter
  unsigned long long v[6] = {n_steps, n_null, n_real, n_esc, n_trunc, n_query};
#pragma unroll
  for (int q = 0; q < 6; q++) {
    unsigned long long x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0 && x) atomicAdd(A.stats + q, x);
  }
}

// ---------------------------------------------------------------- deferred light rays
// Offsets of the tracing blocks' light rays in one list (exclusive sum of
// their counts, in order; off[nb] = the total).
__global__ void k_light_offsets(const uint32_t* __restrict__ cnt, int nb, uint32_t* __restrict__ off) {
  if (threadIdx.x != 0) return;
  uint32_t s = 0;
  for (int b = 0; b < nb; b++) {
    off[b] = s;
    s += cnt[b];
  }
  off[nb] = s;
}

// Bits 0..15 of x to the even bit positions.
__device__ inline uint32_t spread_bits2(uint32_t x) {
  x &= 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Sort keys of the light rays: every ray walks along the sun direction d,
// so rays whose starts project to nearby points of the plane normal to d
// cross the same column of tets.  With (u, v) the start's coordinates in
// that plane and w its coordinate along d (all about the cube's centre,
// mapped from [-0.87, 0.87] to [0, 1)), the 32-bit key is the Z-order of
// (u, v) at cbits bits each (a column bundle), then w at kDepthBits bits,
// then the Z-order of the position within the bundle (fbits bits each).
// Rays of one wave start close together at one depth (walks of similar
// length), and the waves in flight together cover a compact set of
// bundles, whose records stay in the caches.
constexpr int kDepthBits = 10;

__device__ inline uint32_t light_key(float3 p, float3 d, float3 t1, float3 t2, int cbits, int fbits) {
  const float3 c = make_float3(p.x - 0.5f, p.y - 0.5f, p.z - 0.5f);
  const float cu = (c.x * t1.x + c.y * t1.y) + c.z * t1.z;
  const float cv = (c.x * t2.x + c.y * t2.y) + c.z * t2.z;
  const float cw = (c.x * d.x + c.y * d.y) + c.z * d.z;
  auto quant = [](float x, int bits) {
    float f = (x + 0.87f) * (1.0f / 1.74f);
    f = f < 0.0f ? 0.0f : (f > 0.99999f ? 0.99999f : f);
    return (uint32_t)(f * (float)(1u << bits));
  };
  const uint32_t uq = quant(cu, cbits + fbits), vq = quant(cv, cbits + fbits), wq = quant(cw, kDepthBits);
  const uint32_t fm = (1u << fbits) - 1u;
  const uint32_t bundle = spread_bits2(uq >> fbits) | (spread_bits2(vq >> fbits) << 1);
  const uint32_t fine = spread_bits2(uq & fm) | (spread_bits2(vq & fm) << 1);
  return (bundle << (kDepthBits + 2 * fbits)) | (wq << (2 * fbits)) | fine;
}

// Keys and queue positions of the light rays of tracing block blockIdx.x,
// listed from its offset, for the sort.
__global__ void k_light_keys(const LightRec* __restrict__ lq, uint32_t region, const uint32_t* __restrict__ cnt,
                             const uint32_t* __restrict__ off, uint32_t* __restrict__ keys, uint32_t* __restrict__ idx,
                             float3 d, int cbits, int fbits) {
  const uint32_t b = blockIdx.x, n = cnt[b], o = off[b];
  // an orthonormal basis (t1, t2) of the plane normal to d (Duff et al. 2017)
  const float sg = copysignf(1.0f, d.z);
  const float a = -1.0f / (sg + d.z);
  const float bxy = (d.x * d.y) * a;
  const float3 t1 = make_float3(1.0f + ((sg * d.x) * d.x) * a, sg * bxy, -sg * d.x);
  const float3 t2 = make_float3(bxy, sg + (d.y * d.y) * a, -d.y);
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t q = b * region + j;
    const LightRec r = lq[q];
    keys[o + j] = light_key(make_float3(r.x, r.y, r.z), d, t1, t2, cbits, fbits);
    idx[o + j] = q;
  }
}

// The queued light rays in the order of their keys (light_key): neighbouring
// lanes start close together and walk the same direction through the same
// column of tets, so they read the same records.  Each walks to the grid boundary summing the optical depth
// (analytic transmittance, as the tracer's own light walk), then adds its
// weight times e^-depth to its pixel.  A straight walk meets a tet at most
// once, so the tet count bounds it.
template <class Med>
__global__ __launch_bounds__(256) void k_light(RenderArgs A, Med med, const LightRec* __restrict__ lq,
                                               const uint32_t* __restrict__ order, uint32_t n) {
  __shared__ float s_tab[256 * kTabStride];
  float* tab = s_tab + threadIdx.x * kTabStride;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t steps = 0;
  if (i < n) {
    const LightRec r = lq[order[i]];
    const float3 o = make_float3(r.x, r.y, r.z);
    const float3 d = make_float3(A.sun[0], A.sun[1], A.sun[2]);
    set_segment(tab, o, d, Med::kOriginScale);
    uint32_t cell = r.cell;
    float t = 0.0f, od = 0.0f;
    for (;;) {
      const Step st = med.step(cell, o, d, tab, t);
      steps++;
      if (!st.ok) break;
      od = od + st.sigma * (st.te - t);
      t = st.te;
      if (st.next < 0 || (int64_t)steps > med.n) break;
      cell = (uint32_t)st.next;
    }
    const float Tr = exp_neg(od);
    float* px = A.out + 3 * (size_t)r.pix;
    atomicAdd(px, r.w0 * Tr);
    atomicAdd(px + 1, r.w1 * Tr);
    atomicAdd(px + 2, r.w2 * Tr);
  }
  unsigned long long x = steps;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if (__lane_id() == 0 && x) atomicAdd(A.stats + 0, x);
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
static int cu_count() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                 hipSuccess && n > 0)
      cached = n;
    else
      return 256;
  }
  return cached;
}

constexpr int64_t kMaxEntriesPerPass = 1ll << 25;  // 1 GiB of entry records
constexpr int kMaxTraceBlocks = 8192;               // blocks of one tracing launch with a light-ray queue

// Sort buffers of the deferred light rays (keys and positions, both ways)
// and the sort's own scratch.
struct LightSort {
  uint32_t* keys[2];
  uint32_t* idx[2];
  void* temp;
  size_t temp_bytes;
  int cbits, fbits;  // key layout (light_key)
  int64_t queued;    // light rays walked from the queue so far
};

// The pass's queued light rays: their count, the sort by key, the walks.
template <class Med>
static int walk_light_queue(const Med& med, const RenderArgs& P, int nblocks, LightSort& ls, hipStream_t st) {
  uint32_t* off = P.lq_count + kMaxTraceBlocks;
  hipLaunchKernelGGL(k_light_offsets, dim3(1), dim3(64), 0, st, (const uint32_t*)P.lq_count, nblocks, off);
  uint32_t n = 0;
  TV_HIP(hipMemcpyAsync(&n, off + nblocks, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  ls.queued += n;
  if (!n) return TET_OK;
  hipLaunchKernelGGL(k_light_keys, dim3((unsigned)nblocks), dim3(256), 0, st, (const LightRec*)P.lq, P.lq_region,
                     (const uint32_t*)P.lq_count, (const uint32_t*)off, ls.keys[0], ls.idx[0],
                     make_float3(P.sun[0], P.sun[1], P.sun[2]), ls.cbits, ls.fbits);
  size_t tb = ls.temp_bytes;
  if (rocprim::radix_sort_pairs(ls.temp, tb, ls.keys[0], ls.keys[1], ls.idx[0], ls.idx[1], n, 0u, 32u, st) !=
      hipSuccess)
    return fail(TET_ERR_DEVICE, "render: sort of the light rays");
  hipLaunchKernelGGL(k_light<Med>, dim3((n + 255) / 256), dim3(256), 0, st, P, med, (const LightRec*)P.lq,
                     (const uint32_t*)ls.idx[1], n);
  TV_HIP(hipGetLastError());
  return TET_OK;
}

template <class Med, int NRC>
static int run_passes(const Med& med, RenderArgs& A, const tet_render_opts& o, int32_t spp, int64_t npix,
                      char* sc, RayEntry* entries, int64_t pass_cap, hipStream_t st, float* ms_total,
                      float* ms_trace, float* ms_cache, bool timed = true, LightSort* ls = nullptr) {
  if (A.defer && !ls) return fail(TET_ERR_INTERNAL, "render: light-ray queue without its sort");
  int bs = o.block_size ? o.block_size : 256;
  int bpc = o.blocks_per_cu ? o.blocks_per_cu : 8;
  const bool ext = A.ex.model != 0 || A.ex.ch_t || A.ex.ch_a || A.ex.ch_g;
  // timed: HIP events around the passes, waited for after each pass;
  // untimed: kernel launches on the stream only
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, t0 = nullptr, t1 = nullptr;
  struct Ev {
    hipEvent_t *a, *b, *c, *d, *f;
    ~Ev() {
      for (hipEvent_t* e : {a, b, c, d, f})
        if (*e) (void)hipEventDestroy(*e);
    }
  } ev{&e0, &e1, &e2, &t0, &t1};
  if (timed) {
    TV_HIP(hipEventCreate(&e0));
    TV_HIP(hipEventCreate(&e1));
    TV_HIP(hipEventCreate(&e2));
    TV_HIP(hipEventCreate(&t0));
    TV_HIP(hipEventCreate(&t1));
  }
  *ms_total = 0.0f;
  *ms_trace = 0.0f;
  *ms_cache = 0.0f;
  if (timed) TV_HIP(hipEventRecord(e0, st));
  if (A.accumulate && NRC != 2)
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((npix * 3 + 255) / 256)), dim3(256), 0, st, A.out, npix * 3);
  for (int32_t done = 0; done < spp; done += (int32_t)pass_cap) {
    A.pass_start = A.pass_start + (done ? (int32_t)pass_cap : 0);
    A.pass_spp = (int32_t)std::min<int64_t>(pass_cap, spp - done);
    int32_t per = std::min(A.per_item, A.pass_spp);
    int32_t ipp = (A.pass_spp + per - 1) / per;
    RenderArgs P = A;
    P.per_item = per;
    P.items_per_pixel = ipp;
    P.train_items = (NRC == 1 && done == 0) ? A.train_items : 0u;  // training paths ride the first pass
    P.items = A.slots * (uint32_t)ipp + P.train_items;
    P.entries = entries;
    P.range_size = (P.items + 7) / 8;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (uint32_t*)sc, 9);  // ranges, query count
    uint64_t ne = (uint64_t)A.slots * (uint64_t)P.pass_spp;
    hipLaunchKernelGGL(k_raygen<Med>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, P, med, entries);
    if (P.train_items) {  // entry records of the training paths, after the image's
      RenderArgs T = P;
      T.train = 1;
      T.seed = A.train_seed;
      T.slots = P.train_items;
      T.pass_spp = 1;
      hipLaunchKernelGGL(k_raygen<Med>, dim3((P.train_items + 255) / 256), dim3(256), 0, st, T, med,
                         entries + A.train_ent0);
    }
    int64_t grid = (int64_t)cu_count() * bpc;
    int64_t need = ((int64_t)P.items + bs - 1) / bs;
    grid = std::max<int64_t>(1, std::min(grid, need));
    if (A.defer) {  // one queue region per block
      grid = std::min<int64_t>(grid, kMaxTraceBlocks);
      P.lq_region = (uint32_t)(A.lq_cap / (uint64_t)grid);
    }
    if (timed) TV_HIP(hipEventRecord(t0, st));
    if (NRC != 0) {
      if constexpr (!std::is_same<Med, VoxelMedium>::value) {
        if (ext) hipLaunchKernelGGL((k_render<Med, 5, NRC, false, true>), dim3((unsigned)grid), dim3(bs), 0, st, P, med);
        else hipLaunchKernelGGL((k_render<Med, 5, NRC>), dim3((unsigned)grid), dim3(bs), 0, st, P, med);
      }
    } else if (ext) {
      if constexpr (!std::is_same<Med, VoxelMedium>::value) {
        switch (o.waves_per_simd) {
          case 4: hipLaunchKernelGGL((k_render<Med, 4, 0, false, true>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
          case 6: hipLaunchKernelGGL((k_render<Med, 6, 0, false, true>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
          case 8: hipLaunchKernelGGL((k_render<Med, 8, 0, false, true>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
          default: hipLaunchKernelGGL((k_render<Med, 5, 0, false, true>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
        }
      }
    } else {
      switch (o.waves_per_simd) {
        case 4: hipLaunchKernelGGL((k_render<Med, 4, 0>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
        case 6: hipLaunchKernelGGL((k_render<Med, 6, 0>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
        case 8: hipLaunchKernelGGL((k_render<Med, 8, 0>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
        default: hipLaunchKernelGGL((k_render<Med, 5, 0>), dim3((unsigned)grid), dim3(bs), 0, st, P, med); break;
      }
    }
    TV_HIP(hipGetLastError());
    if constexpr (NRC != 2 && !std::is_same<Med, VoxelMedium>::value) {
      if (A.defer && ls)  // the pass's queued light rays, part of the tracing time
        if (int rc = walk_light_queue(med, P, (int)grid, *ls, st)) return rc;
    }
    if (timed) TV_HIP(hipEventRecord(t1, st));
    if (NRC == 1)  // the pass's cache queries, added to their pixels
      if (int rc = nrc_query_pass(A.nrc, A.qbuf, A.qpix, A.qcount, A.out, (int64_t)ne, st)) return rc;
    if (timed) {
      TV_HIP(hipEventRecord(e2, st));
      TV_HIP(hipEventSynchronize(e2));
      float ms = 0.0f;
      TV_HIP(hipEventElapsedTime(&ms, t0, t1));
      *ms_trace += ms;
      TV_HIP(hipEventElapsedTime(&ms, t1, e2));
      *ms_cache += ms;
    }
  }
  if (A.accumulate && NRC != 2)
    hipLaunchKernelGGL(k_scale_f32, dim3((unsigned)((npix * 3 + 255) / 256)), dim3(256), 0, st, A.out, npix * 3,
                       (float)spp);
  TV_HIP(hipGetLastError());
  if (timed) {
    TV_HIP(hipEventRecord(e1, st));
    TV_HIP(hipEventSynchronize(e1));
    TV_HIP(hipEventElapsedTime(ms_total, e0, e1));
  }
  return TET_OK;
}

static int check_render_opts(const tet_render_opts& o) {
  if (o.max_bounces < 1 || o.transmittance < 0 || o.transmittance > 2 || o.max_steps_per_path < 1 ||
      o.sample_offset < 0 || o.samples_per_item < 0 || o.block_size < 0 || o.block_size > 256 ||
      (o.block_size % 64) != 0 || o.blocks_per_cu < 0 ||
      (o.waves_per_simd != 0 && o.waves_per_simd != 4 && o.waves_per_simd != 5 && o.waves_per_simd != 6 &&
       o.waves_per_simd != 8) ||
      (o.record_layout != 0 && o.record_layout != 32 && o.record_layout != 48) || o.batch_items < 0 ||
      o.batch_items > (1 << 20) || o.event_wait < 0 || o.event_wait > 64)
    return fail(TET_ERR_INVALID_ARG, "render: bad options");
  return TET_OK;
}

static void set_scene(RenderArgs& A, const tet_camera* cam, const tet_medium* medm, const tet_light* light) {
  make_frame(*cam, &A.fr);
  A.albedo = medm->albedo;
  A.g = medm->g;
  for (int i = 0; i < 3; i++) {
    A.sun[i] = light->sun_dir[i];
    A.E[i] = light->sun_irradiance[i];
    A.env[i] = light->env_radiance[i];
  }
}

// Extra channels (temperature, albedo, phase parameter per tet): a tet grid
// that carries at least one, and a finite emission colour >= 0.  They
// combine with the radiance cache (the cache at a vertex stands for all the
// radiance from it on, the vertex's emission included).
static int check_channels(const tet_render_opts& o, const tet_grid* g, const char* who) {
  if (!o.channels) return TET_OK;
  const std::string w(who);
  if (o.channels != 1) return fail(TET_ERR_INVALID_ARG, w + ": channels must be 0 or 1");
  if (!g) return fail(TET_ERR_UNSUPPORTED, w + ": channels need a tet grid");
  if (!g->ch[0] && !g->ch[1] && !g->ch[2]) return fail(TET_ERR_INVALID_ARG, w + ": the grid has no channels");
  for (int c = 0; c < 3; c++)
    if (!(o.emission[c] >= 0.0f) || std::isinf(o.emission[c]))
      return fail(TET_ERR_INVALID_ARG, w + ": emission must be finite and >= 0");
  return TET_OK;
}

// The voxel-lookup model has no analytic light transmittance.
static int check_model(const tet_render_opts& o, const tet_grid* g, const char* who) {
  if (g && g->model == 2 && o.transmittance == 0)
    return fail(TET_ERR_INVALID_ARG,
                std::string(who) + ": the voxel-lookup model needs ratio or delta tracking for the light");
  return TET_OK;
}

// The channels (when asked for) and the density model of grid g.
static void set_ext(ExtArgs& X, const tet_grid* g, const tet_render_opts& o) {
  memset(&X, 0, sizeof(X));
  if (o.channels) {
    X.ch_t = g->ch[0];
    X.ch_a = g->ch[1];
    X.ch_g = g->ch[2];
    for (int c = 0; c < 3; c++) X.emission[c] = o.emission[c];
  }
  if (g->model) {
    X.model = g->model;
    X.mcoef = g->mcoef;
    X.mdens = g->mdens;
    X.mn = g->mn;
    X.mscale = g->mscale;
  }
}

static int render_common(int kind, const tet_grid* g, const tet_density* dens, const tet_camera* cam,
                         const tet_medium* medm, const tet_light* light, int32_t spp, uint64_t seed,
                         const tet_render_opts* opts_in, float* out_rgb, int32_t on_device, hipStream_t st,
                         tet_render_stats* stats, char* fixed = nullptr, size_t fixed_bytes = 0) {
  // fixed != NULL: the scratch is the caller's fixed device array (no
  // allocation, no timing, no wait; launches on the stream only)
  const bool noalloc = fixed != nullptr;
  if (int rc = check_camera(cam)) return rc;
  if (!medm || !light || !out_rgb) return fail(TET_ERR_INVALID_ARG, "render: NULL medium, light or output");
  if (spp < 1) return fail(TET_ERR_INVALID_ARG, "render: spp must be >= 1");
  if (!(medm->g > -1.0f && medm->g < 1.0f) || !(medm->albedo >= 0.0f))
    return fail(TET_ERR_INVALID_ARG, "render: medium needs albedo >= 0 and -1 < g < 1");
  tet_render_opts o;
  if (opts_in) o = *opts_in;
  else tet_render_opts_defaults(&o);
  if (int rc = check_render_opts(o)) return rc;
  const tet_nrc* nrc = o.nrc;
  if (nrc && kind != 0) return fail(TET_ERR_UNSUPPORTED, "render: the radiance cache needs a tet grid");
  const bool train = nrc && o.nrc_train;
  const int32_t n_train = train ? nrc->opts.train_paths : 0, kv = train ? nrc->opts.train_vertices : 0;
  if (train)
    if (int rc = nrc_resolve_sigma_ref(const_cast<tet_nrc*>(nrc), g, st)) return rc;
  if (nrc && !(nrc->opts.sigma_ref > 0.0f))
    return fail(TET_ERR_INVALID_ARG, "render: the radiance cache has no sigma_ref yet (train it or set one)");
  if ((int64_t)o.sample_offset + spp > (1ll << 31)) return fail(TET_ERR_INVALID_ARG, "render: sample range too large");
  if (int rc = check_channels(o, kind == 0 ? g : nullptr, "render")) return rc;
  if (int rc = check_model(o, kind == 0 ? g : nullptr, "render")) return rc;
  const bool model = kind == 0 && g->model != 0;  // walk the records whose majorants bound the model
  if (noalloc && (kind != 0 || nrc || !on_device || stats))
    return fail(TET_ERR_UNSUPPORTED,
                "tet_render_noalloc: tet grids only, no radiance cache, output on the device, no stats");
  // the no-alloc path only takes a shape table that already exists (every
  // grid's build made the one of its device)
  const uint32_t* shapes = noalloc ? shape_table_existing() : shape_table();
  if (!shapes) return fail(TET_ERR_DEVICE, "render: shape table");
  int64_t npix = (int64_t)cam->width * cam->height;
  int tiles_x = (cam->width + 7) / 8, tiles_y = (cam->height + 7) / 8;
  int64_t slots = (int64_t)tiles_x * tiles_y * 64;
  if (slots >= (1ll << 31)) return fail(TET_ERR_INVALID_ARG, "render: image too large");
  const int64_t entry_cap =
      noalloc ? std::min<int64_t>(kMaxEntriesPerPass, ((int64_t)fixed_bytes - 256) / (int64_t)sizeof(RayEntry))
              : kMaxEntriesPerPass;
  if (noalloc && slots > entry_cap)
    return fail(TET_ERR_CAPACITY, "tet_render_noalloc: one sample per pixel of this image does not fit the "
                                  "fixed scratch (" + std::to_string(entry_cap) + " entry records)");
  int64_t pass_cap = std::max<int64_t>(1, std::min<int64_t>(spp, entry_cap / slots));
  int per_item = (o.samples_per_item <= 0 || o.samples_per_item > pass_cap) ? (int)pass_cap : o.samples_per_item;
  if (slots * ((pass_cap + per_item - 1) / per_item) >= (1ll << 32))
    return fail(TET_ERR_INVALID_ARG, "render: too many work items");

  RenderArgs A;
  memset(&A, 0, sizeof(A));
  set_scene(A, cam, medm, light);
  if (kind == 0) set_ext(A.ex, g, o);
  A.spp = spp;
  A.pass_start = o.sample_offset;
  A.per_item = per_item;
  A.max_bounces = o.max_bounces;
  A.transmittance = o.transmittance;
  A.max_steps = (uint32_t)std::min<int64_t>(o.max_steps_per_path, 0x7FFFFFFF);
  A.seed = seed;
  A.slots = (uint32_t)slots;
  A.tiles_x = tiles_x;
  A.batch = o.batch_items ? (uint32_t)o.batch_items : 64u;
  A.event_wait = o.event_wait ? o.event_wait : 32;
  // Light rays are queued and walked after each pass, sorted by start tet,
  // on tet grids without a density model (channels and the radiance cache's
  // renders included) with analytic light transmittance when the step
  // guard is at its largest value (2^31 - 1: each light walk then runs on its
  // own, bounded by the tet count, while the guard would count all of a
  // path's walks together; the estimate is the same unless a path takes
  // more than 2^31 - 1 steps).  Their terms are added to the pixels apart
  // from the rest of their samples.
  const bool defer = kind == 0 && !model && !noalloc && o.transmittance == 0 && o.max_steps_per_path >= 0x7FFFFFFF;
  A.accumulate = (pass_cap < spp) || (per_item < pass_cap) || nrc != nullptr || defer;
  if (nrc) {
    A.nrc = nrc;
    A.truncate = nrc->opts.truncate_bounce;
  }
  if (train) {
    A.train_items = (uint32_t)n_train;
    A.train_ent0 = (uint32_t)(slots * pass_cap);
    A.train_seed = seed ^ 0x6A09E667F3BCC909ull;
    A.npix = (uint32_t)npix;
    A.rec_vertices = kv;
  }

  // scratch: counters, entry records of one pass (then those of the training
  // paths), image when the output is on the host, training-path records
  size_t img_bytes = (size_t)npix * 3 * sizeof(float);
  size_t ent_bytes = ((size_t)slots * (size_t)pass_cap + (size_t)n_train) * sizeof(RayEntry);
  size_t vrec_bytes = (size_t)n_train * (size_t)kv * 48, pl_bytes = (size_t)n_train * 16;
  size_t q_bytes = nrc ? (size_t)slots * (size_t)pass_cap * 36 : 0;  // at most one query per sample
  size_t scratch = 256 + ent_bytes + (on_device ? 0 : img_bytes) + vrec_bytes + pl_bytes + q_bytes;
  if (noalloc && scratch > fixed_bytes) return fail(TET_ERR_INTERNAL, "tet_render_noalloc: scratch overrun");
  char* sc = noalloc ? fixed : (char*)dev_alloc(scratch);
  if (!sc) return fail(TET_ERR_OUT_OF_MEMORY, "render: scratch");
  struct Free {
    void* p;
    ~Free() { if (p) dev_free(p); }
  } fr_{noalloc ? nullptr : sc};
  A.counter = (uint32_t*)sc;
  A.stats = (unsigned long long*)(sc + 64);  // counters: 8 work ranges in sc[0..32), query count at sc[32]
  RayEntry* entries = (RayEntry*)(sc + 256);
  A.out = on_device ? out_rgb : (float*)(sc + 256 + ent_bytes);
  if (train) {
    char* tr = sc + 256 + ent_bytes + (on_device ? 0 : img_bytes);
    A.vrec = (float4*)tr;
    A.path_l = (float4*)(tr + vrec_bytes);
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (uint32_t*)sc, 64);

  // the light-ray queue of a pass (at most 4 light rays per sample, 2^26 in
  // all; a full queue leaves the rest to the tracing lanes) and its sort
  LightSort ls;
  memset(&ls, 0, sizeof(ls));
  struct FreeQ {
    void* p;
    ~FreeQ() { if (p) dev_free(p); }
  } frq_{nullptr};
  if (defer) {
    const uint32_t cap = (uint32_t)std::min<int64_t>(1ll << 26, std::max<int64_t>(1024, slots * pass_cap * 4));
    // column bundles about as wide as the grid's typical tet: bits per
    // axis ~ log2(tets) / 3 (8 on a 7 M-tet grid, 9 on 86 M tets)
    int tet_bits = 0;
    while (tet_bits < 40 && (int64_t)(1ull << tet_bits) < g->n) tet_bits++;
    ls.cbits = std::max(4, std::min(11, (tet_bits + 1) / 3));
    ls.fbits = (32 - kDepthBits - 2 * ls.cbits) / 2;
    if (rocprim::radix_sort_pairs(nullptr, ls.temp_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, cap, 0u, 32u, st) != hipSuccess)
      return fail(TET_ERR_DEVICE, "render: light-ray sort size");
    const size_t head = (size_t)(2 * kMaxTraceBlocks + 64) * 4;  // per-block counts, then their offsets
    const size_t qb = head + (size_t)cap * sizeof(LightRec) + 4 * (size_t)cap * 4 + ((ls.temp_bytes + 255) & ~size_t(255));
    char* q = (char*)dev_alloc(qb);
    if (!q) return fail(TET_ERR_OUT_OF_MEMORY, "render: light-ray queue");
    frq_.p = q;
    A.defer = 1;
    A.lq_count = (uint32_t*)q;
    A.lq_cap = cap;
    A.lq = (LightRec*)(q + head);
    uint32_t* k = (uint32_t*)(q + head + (size_t)cap * sizeof(LightRec));
    ls.keys[0] = k;
    ls.keys[1] = k + cap;
    ls.idx[0] = k + 2 * (size_t)cap;
    ls.idx[1] = k + 3 * (size_t)cap;
    ls.temp = k + 4 * (size_t)cap;
  }

  if (nrc) {
    char* qb = sc + 256 + ent_bytes + (on_device ? 0 : img_bytes) + vrec_bytes + pl_bytes;
    A.qbuf = (float4*)qb;
    A.qpix = (uint32_t*)(qb + (size_t)slots * (size_t)pass_cap * 32);
    A.qcount = (uint32_t*)sc + 8;
  }
  float ms = 0.0f, ms_trace = 0.0f, ms_cache = 0.0f;
  int rc;
  if (kind == 0 && g->rec32 && o.record_layout != 48) {
    TetMedium32 m{model ? g->mrec32 : g->rec32, g->keys, g->n, g->max_depth, shapes, g->kidx, g->kbits};
    rc = nrc ? run_passes<TetMedium32, 1>(m, A, o, spp, npix, sc, entries, pass_cap, st, &ms, &ms_trace, &ms_cache,
                                          !noalloc, &ls)
             : run_passes<TetMedium32, 0>(m, A, o, spp, npix, sc, entries, pass_cap, st, &ms, &ms_trace, &ms_cache,
                                          !noalloc, &ls);
  } else if (kind == 0) {
    if (o.record_layout == 32) return fail(TET_ERR_UNSUPPORTED, "render: this grid has no compact records");
    TetMedium m{model ? g->mrec : g->rec, g->keys, g->n, g->max_depth, shapes, g->kidx, g->kbits};
    rc = nrc ? run_passes<TetMedium, 1>(m, A, o, spp, npix, sc, entries, pass_cap, st, &ms, &ms_trace, &ms_cache,
                                        !noalloc, &ls)
             : run_passes<TetMedium, 0>(m, A, o, spp, npix, sc, entries, pass_cap, st, &ms, &ms_trace, &ms_cache,
                                        !noalloc, &ls);
  } else {
    VoxelMedium m{dens->data, dens->n, dens->density_scale};
    rc = run_passes<VoxelMedium, 0>(m, A, o, spp, npix, sc, entries, pass_cap, st, &ms, &ms_trace, &ms_cache,
                                    !noalloc);
  }
  if (rc) return rc;
  if (noalloc) return TET_OK;
  int64_t records = 0;
  double loss = 0.0;
  if (train) {  // the cache's Adam steps on the frame's training paths (timed into ms)
    hipEvent_t t0, t1;
    TV_HIP(hipEventCreate(&t0));
    TV_HIP(hipEventCreate(&t1));
    struct Ev {
      hipEvent_t a, b;
      ~Ev() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } ev{t0, t1};
    TV_HIP(hipEventRecord(t0, st));
    if (int trc = nrc_train_paths(const_cast<tet_nrc*>(nrc), A.vrec, A.path_l, n_train, kv, st, &records, &loss))
      return trc;
    TV_HIP(hipEventRecord(t1, st));
    TV_HIP(hipEventSynchronize(t1));
    float tms = 0.0f;
    TV_HIP(hipEventElapsedTime(&tms, t0, t1));
    ms += tms;
  }
  unsigned long long hs[6] = {0, 0, 0, 0, 0, 0};
  TV_HIP(hipMemcpyAsync(hs, A.stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (!on_device) TV_HIP(hipMemcpyAsync(out_rgb, A.out, img_bytes, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  if (stats) {
    stats->tet_steps = (int64_t)hs[0];
    stats->null_collisions = (int64_t)hs[1];
    stats->real_collisions = (int64_t)hs[2];
    stats->escapes = (int64_t)hs[3];
    stats->truncated = (int64_t)hs[4];
    stats->ms = ms;
    stats->trace_ms = ms_trace;
    stats->cache_ms = ms_cache;
    stats->cache_queries = (int64_t)hs[5];
    stats->cache_records = records;
    stats->cache_loss = loss;
    stats->light_rays_queued = ls.queued;
  }
  return TET_OK;
}

int trace_training_paths(const tet_grid* g, const tet_camera* cam, const tet_medium* medm, const tet_light* light,
                         uint64_t frame_seed, const tet_render_opts* opts_in, int32_t n_paths, int32_t kv, float4* vrec,
                         float4* path_l, hipStream_t st, float* ms_out) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "training paths: grid is NULL");
  const uint32_t* shapes = shape_table();
  if (!shapes) return fail(TET_ERR_DEVICE, "training paths: shape table");
  if (int rc = check_camera(cam)) return rc;
  if (!medm || !light) return fail(TET_ERR_INVALID_ARG, "training paths: NULL medium or light");
  if (!(medm->g > -1.0f && medm->g < 1.0f) || !(medm->albedo >= 0.0f))
    return fail(TET_ERR_INVALID_ARG, "training paths: medium needs albedo >= 0 and -1 < g < 1");
  tet_render_opts o;
  if (opts_in) o = *opts_in;
  else tet_render_opts_defaults(&o);
  if (int rc = check_render_opts(o)) return rc;
  if (int rc = check_channels(o, g, "training paths")) return rc;
  if (int rc = check_model(o, g, "training paths")) return rc;
  if (n_paths < 1 || kv < 1) return fail(TET_ERR_INVALID_ARG, "training paths: bad counts");
  RenderArgs A;
  memset(&A, 0, sizeof(A));
  set_scene(A, cam, medm, light);
  set_ext(A.ex, g, o);
  A.spp = 1;
  A.per_item = 1;
  A.max_bounces = o.max_bounces;
  A.transmittance = o.transmittance;
  A.max_steps = (uint32_t)std::min<int64_t>(o.max_steps_per_path, 0x7FFFFFFF);
  A.seed = frame_seed;
  A.slots = (uint32_t)n_paths;
  A.tiles_x = (cam->width + 7) / 8;
  A.batch = o.batch_items ? (uint32_t)o.batch_items : 64u;
  A.event_wait = o.event_wait ? o.event_wait : 48;
  A.train = 1;
  A.npix = (uint32_t)((int64_t)cam->width * cam->height);
  A.rec_vertices = kv;
  A.vrec = vrec;
  A.path_l = path_l;
  size_t ent_bytes = (size_t)n_paths * sizeof(RayEntry);
  char* sc = (char*)dev_alloc(256 + ent_bytes);
  if (!sc) return fail(TET_ERR_OUT_OF_MEMORY, "training paths: scratch");
  struct Free {
    void* p;
    ~Free() { dev_free(p); }
  } fr_{sc};
  A.counter = (uint32_t*)sc;
  A.stats = (unsigned long long*)(sc + 64);
  RayEntry* entries = (RayEntry*)(sc + 256);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (uint32_t*)sc, 64);
  float ms = 0.0f, ms_trace = 0.0f, ms_cache = 0.0f;
  int rc;
  const bool model = g->model != 0;
  if (g->rec32 && o.record_layout != 48) {
    TetMedium32 m{model ? g->mrec32 : g->rec32, g->keys, g->n, g->max_depth, shapes, g->kidx, g->kbits};
    rc = run_passes<TetMedium32, 2>(m, A, o, 1, 0, sc, entries, 1, st, &ms, &ms_trace, &ms_cache);
  } else {
    if (o.record_layout == 32) return fail(TET_ERR_UNSUPPORTED, "training paths: this grid has no compact records");
    TetMedium m{model ? g->mrec : g->rec, g->keys, g->n, g->max_depth, shapes, g->kidx, g->kbits};
    rc = run_passes<TetMedium, 2>(m, A, o, 1, 0, sc, entries, 1, st, &ms, &ms_trace, &ms_cache);
  }
  if (rc) return rc;
  TV_HIP(hipStreamSynchronize(st));
  if (ms_out) *ms_out = ms_trace;
  return TET_OK;
}

int render_grid(const tet_grid* g, const tet_camera* cam, const tet_medium* m, const tet_light* l, int32_t spp,
                uint64_t seed, const tet_render_opts* o, float* out, int32_t on_device, hipStream_t st,
                tet_render_stats* stats) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_render: grid is NULL");
  return render_common(0, g, nullptr, cam, m, l, spp, seed, o, out, on_device, st, stats);
}

// ---------------------------------------------------------------- render without allocation
// The scratch of tet_render_noalloc: a fixed array, one copy per device (made
// when the library's code is loaded on it, kept until the process ends).  In
// host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, looked up once per device.
constexpr size_t kNoAllocBytes = (size_t(64) << 20) + 256;  // counters, then 2^21 entry records
static __device__ __align__(256) char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;

static char* noalloc_scratch() {
  static std::mutex mu;
  static char* ptr[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptr[dev] = (char*)p;
  }
  return ptr[dev];
}

int render_grid_noalloc(const tet_grid* g, const tet_camera* cam, const tet_medium* m, const tet_light* l,
                        int32_t spp, uint64_t seed, const tet_render_opts* o, float* out, hipStream_t st) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_render_noalloc: grid is NULL");
  int dev = -1;
  TV_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(TET_ERR_INVALID_ARG, "tet_render_noalloc: the grid lives on another device");
  char* sc = noalloc_scratch();
  if (!sc) return fail(TET_ERR_DEVICE, "tet_render_noalloc: no device address for the fixed scratch");
  return render_common(0, g, nullptr, cam, m, l, spp, seed, o, out, 1, st, nullptr, sc, kNoAllocBytes);
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

// ---------------------------------------------------------------- batches of scenes
struct BatchState {
  int device = 0;
  int n = 0;
  bool use32 = true;
  bool ext = false;  // some scene carries channels or a density model
  const uint32_t* shapes = nullptr;
  tet_render_opts o;
  SceneDesc* pinned = nullptr;  // host staging of the scene table (page-locked)
  SceneDesc* table = nullptr;   // device scene table
  char* scratch = nullptr;      // counters and statistics, then the entry records
  RenderArgs A;
  uint64_t total_px = 0;
  int grid = 1, bs = 256;
  hipStream_t cap = nullptr;    // capture stream of the frame graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchState() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    dev_free(table);
    dev_free(scratch);
    if (pinned) (void)hipHostFree(pinned);
  }
};

static int batch_setup(BatchState* B, int32_t n, const tet_grid* const* grids, const tet_camera* cams,
                       const tet_medium* media, const tet_light* lights, const int32_t* spp,
                       const tet_render_opts* opts_in, float* const* outs) {
  if (n < 1 || n > 4096 || !grids || !cams || !media || !lights || !spp || !outs)
    return fail(TET_ERR_INVALID_ARG, "render batch: bad arguments (1 <= n <= 4096, no NULL arrays)");
  tet_render_opts o;
  if (opts_in) o = *opts_in;
  else tet_render_opts_defaults(&o);
  if (int rc = check_render_opts(o)) return rc;
  if (o.nrc) return fail(TET_ERR_UNSUPPORTED, "render batch: no radiance cache in batches");
  bool use32 = o.record_layout != 48;
  for (int i = 0; i < n; i++) {
    if (!grids[i] || !outs[i]) return fail(TET_ERR_INVALID_ARG, "render batch: NULL grid or output");
    if (int rc = check_channels(o, grids[i], "render batch")) return rc;
    if (int rc = check_model(o, grids[i], "render batch")) return rc;
    if (int rc = check_camera(&cams[i])) return rc;
    if (!(media[i].g > -1.0f && media[i].g < 1.0f) || !(media[i].albedo >= 0.0f))
      return fail(TET_ERR_INVALID_ARG, "render batch: medium needs albedo >= 0 and -1 < g < 1");
    if (spp[i] < 1 || (int64_t)o.sample_offset + spp[i] > (1ll << 31))
      return fail(TET_ERR_INVALID_ARG, "render batch: bad spp");
    if (!grids[i]->rec32) use32 = false;
  }
  if (!use32 && o.record_layout == 32)
    return fail(TET_ERR_UNSUPPORTED, "render batch: a grid has no compact records");
  B->n = n;
  B->o = o;
  B->use32 = use32;
  B->shapes = shape_table();  // made here: a captured frame cannot upload it
  if (!B->shapes) return fail(TET_ERR_DEVICE, "render batch: shape table");
  if (hipGetDevice(&B->device) != hipSuccess) return fail(TET_ERR_DEVICE, "render batch: no device");
  std::vector<SceneDesc> host((size_t)n);
  uint64_t item = 0, entry = 0, px = 0;
  for (int i = 0; i < n; i++) {
    SceneDesc& S = host[i];
    memset(&S, 0, sizeof(S));
    make_frame(cams[i], &S.fr);
    S.albedo = media[i].albedo;
    S.g = media[i].g;
    for (int c = 0; c < 3; c++) {
      S.sun[c] = lights[i].sun_dir[c];
      S.E[c] = lights[i].sun_irradiance[c];
      S.env[c] = lights[i].env_radiance[c];
    }
    S.spp = spp[i];
    S.tiles_x = (cams[i].width + 7) / 8;
    int64_t tiles_y = (cams[i].height + 7) / 8;
    uint64_t items = (uint64_t)S.tiles_x * (uint64_t)tiles_y * 64ull * (uint64_t)spp[i];
    S.s0 = (uint32_t)o.sample_offset;
    S.items = (uint32_t)std::min<uint64_t>(items, 0xFFFFFFFFull);
    S.item0 = (uint32_t)std::min<uint64_t>(item, 0xFFFFFFFFull);
    S.entry0 = entry;
    S.pix0 = px;
    const tet_grid* g = grids[i];
    if (g->model) S.rec = use32 ? (const void*)g->mrec32 : (const void*)g->mrec;
    else S.rec = use32 ? (const void*)g->rec32 : (const void*)g->rec;
    set_ext(S.ex, g, o);
    if (o.channels || g->model) B->ext = true;
    S.keys = g->keys;
    S.kidx = g->kidx;
    S.kbits = g->kbits;
    S.n = g->n;
    S.dmax = g->max_depth;
    S.out = outs[i];
    item += (items + 63) / 64 * 64;
    entry += items;
    px += (uint64_t)cams[i].width * (uint64_t)cams[i].height;
    if (items >= (1ull << 32) || item >= (1ull << 32) || entry >= (1ull << 32))
      return fail(TET_ERR_INVALID_ARG, "render batch: more than 2^32 samples in one batch");
  }
  B->total_px = px;
  B->table = (SceneDesc*)dev_alloc(sizeof(SceneDesc) * (size_t)n);
  B->scratch = (char*)dev_alloc(256 + (size_t)entry * sizeof(RayEntry));
  if (hipHostMalloc((void**)&B->pinned, sizeof(SceneDesc) * (size_t)n, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    B->pinned = nullptr;
  }
  if (!B->table || !B->scratch || !B->pinned) return fail(TET_ERR_OUT_OF_MEMORY, "render batch: device memory");
  memcpy(B->pinned, host.data(), sizeof(SceneDesc) * (size_t)n);
  RenderArgs& A = B->A;
  memset(&A, 0, sizeof(A));
  A.max_bounces = o.max_bounces;
  A.transmittance = o.transmittance;
  A.max_steps = (uint32_t)std::min<int64_t>(o.max_steps_per_path, 0x7FFFFFFF);
  A.per_item = 1;
  A.items = (uint32_t)item;
  A.range_size = (uint32_t)(((item + 7) / 8 + 63) / 64 * 64);
  A.batch = 64;  // a wave's batch stays within one scene (scenes' items are padded to 64)
  A.event_wait = o.event_wait ? o.event_wait : 32;
  A.accumulate = 1;
  A.counter = (uint32_t*)B->scratch;
  A.stats = (unsigned long long*)(B->scratch + 64);
  A.entries = (const RayEntry*)(B->scratch + 256);
  A.scenes = B->table;
  A.nscenes = n;
  A.total_entries = entry;
  B->bs = o.block_size ? o.block_size : 256;
  int bpc = o.blocks_per_cu ? o.blocks_per_cu : 8;
  B->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cu_count() * bpc, ((int64_t)item + B->bs - 1) / B->bs));
  return TET_OK;
}

// The frame's kernels (no host synchronisation, no memset: capturable).
static int batch_enqueue(const BatchState* B, hipStream_t st) {
  const RenderArgs& A = B->A;
  RayEntry* entries = (RayEntry*)(B->scratch + 256);
  unsigned pblocks = (unsigned)((B->total_px + 255) / 256);
  unsigned eblocks = (unsigned)((A.total_entries + 255) / 256);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, (uint32_t*)B->scratch, 64);
  hipLaunchKernelGGL(k_batch_images, dim3(pblocks), dim3(256), 0, st, (const SceneDesc*)B->table, B->n, B->total_px, 1);
  if (B->use32) {
    TetMedium32 m{nullptr, nullptr, 0, 0, B->shapes, nullptr, 0};
    hipLaunchKernelGGL(k_raygen_batch<TetMedium32>, dim3(eblocks), dim3(256), 0, st, A, m, entries);
    if (B->ext) hipLaunchKernelGGL((k_render<TetMedium32, 5, 0, true, true>), dim3((unsigned)B->grid), dim3(B->bs), 0, st, A, m);
    else hipLaunchKernelGGL((k_render<TetMedium32, 5, 0, true>), dim3((unsigned)B->grid), dim3(B->bs), 0, st, A, m);
  } else {
    TetMedium m{nullptr, nullptr, 0, 0, B->shapes, nullptr, 0};
    hipLaunchKernelGGL(k_raygen_batch<TetMedium>, dim3(eblocks), dim3(256), 0, st, A, m, entries);
    if (B->ext) hipLaunchKernelGGL((k_render<TetMedium, 5, 0, true, true>), dim3((unsigned)B->grid), dim3(B->bs), 0, st, A, m);
    else hipLaunchKernelGGL((k_render<TetMedium, 5, 0, true>), dim3((unsigned)B->grid), dim3(B->bs), 0, st, A, m);
  }
  hipLaunchKernelGGL(k_batch_images, dim3(pblocks), dim3(256), 0, st, (const SceneDesc*)B->table, B->n, B->total_px, 0);
  TV_HIP(hipGetLastError());
  return TET_OK;
}

// One frame: new seeds into the table, then the kernels (eagerly, or the
// captured graph), then the counters.
static int batch_run(BatchState* B, const uint64_t* seeds, hipStream_t st, tet_render_stats* stats) {
  if (!seeds) return fail(TET_ERR_INVALID_ARG, "render batch: seeds is NULL");
  for (int i = 0; i < B->n; i++) B->pinned[i].seed = seeds[i];
  hipEvent_t e0, e1;
  TV_HIP(hipEventCreate(&e0));
  TV_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  TV_HIP(hipMemcpyAsync(B->table, B->pinned, sizeof(SceneDesc) * (size_t)B->n, hipMemcpyHostToDevice, st));
  TV_HIP(hipEventRecord(e0, st));
  if (B->exec) {
    TV_HIP(hipGraphLaunch(B->exec, st));
  } else if (int rc = batch_enqueue(B, st)) {
    return rc;
  }
  TV_HIP(hipEventRecord(e1, st));
  unsigned long long hs[6] = {0, 0, 0, 0, 0, 0};
  TV_HIP(hipMemcpyAsync(hs, B->A.stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  float ms = 0.0f;
  TV_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->tet_steps = (int64_t)hs[0];
    stats->null_collisions = (int64_t)hs[1];
    stats->real_collisions = (int64_t)hs[2];
    stats->escapes = (int64_t)hs[3];
    stats->truncated = (int64_t)hs[4];
    stats->ms = ms;
    stats->trace_ms = ms;
  }
  return TET_OK;
}

int render_batch(int32_t n, const tet_grid* const* grids, const tet_camera* cams, const tet_medium* media,
                 const tet_light* lights, const int32_t* spp, const uint64_t* seeds, const tet_render_opts* opts,
                 float* const* outs, hipStream_t st, tet_render_stats* stats) {
  BatchState B;
  if (int rc = batch_setup(&B, n, grids, cams, media, lights, spp, opts, outs)) return rc;
  return batch_run(&B, seeds, st, stats);
}

int batch_create(int32_t n, const tet_grid* const* grids, const tet_camera* cams, const tet_medium* media,
                 const tet_light* lights, const int32_t* spp, const tet_render_opts* opts, float* const* outs,
                 void** out) {
  if (!out) return fail(TET_ERR_INVALID_ARG, "tet_batch_create: out is NULL");
  *out = nullptr;
  BatchState* B = new BatchState();
  if (int rc = batch_setup(B, n, grids, cams, media, lights, spp, opts, outs)) {
    delete B;
    return rc;
  }
  // capture the frame's kernels once; frames replay the graph
  hipError_t e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete B;
    return fail(TET_ERR_DEVICE, std::string("tet_batch_create: capture: ") + hipGetErrorString(e));
  }
  int rc = batch_enqueue(B, B->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(B->cap, &g);
  B->graph = g;
  if (rc || e != hipSuccess) {
    delete B;
    return rc ? rc : fail(TET_ERR_DEVICE, std::string("tet_batch_create: capture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    B->exec = nullptr;
    delete B;
    return fail(TET_ERR_DEVICE, std::string("tet_batch_create: instantiate: ") + hipGetErrorString(e));
  }
  *out = B;
  return TET_OK;
}

int batch_render(void* b, const uint64_t* seeds, hipStream_t st, tet_render_stats* stats) {
  if (!b) return fail(TET_ERR_INVALID_ARG, "tet_batch_render: batch is NULL");
  return batch_run((BatchState*)b, seeds, st, stats);
}

void batch_free(void* b) { delete (BatchState*)b; }

int batch_device(const void* b) { return b ? ((const BatchState*)b)->device : 0; }

int locate_points(const tet_grid* g, const float* pts, int64_t count, int64_t* out, int32_t on_device,
                  hipStream_t st) {
  if (!g || count < 0 || (count && (!pts || !out))) return fail(TET_ERR_INVALID_ARG, "tet_locate: bad arguments");
  if (count == 0) return TET_OK;
  const uint32_t* shapes = shape_table();
  if (!shapes) return fail(TET_ERR_DEVICE, "tet_locate: shape table");
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
  TetMedium m{g->rec, g->keys, g->n, g->max_depth, shapes, g->kidx, g->kbits};
  hipLaunchKernelGGL(k_locate, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, m, dp, count, dout);
  TV_HIP(hipGetLastError());
  if (!on_device) TV_HIP(hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

// The tracer's elementary functions at given arguments (fn: 0 -ln(1 - a),
// 1 e^-a, 2 (cos, sin)(2 pi a) into out[2i], out[2i + 1], 3 the HG density
// of cosine a for g = b, 4 the HG inverse CDF at a for g = b).
__global__ void k_eval_functions(int fn, int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                                 float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = a[i];
  switch (fn) {
    case 0: out[i] = exp_tau(x); break;
    case 1: out[i] = exp_neg(x); break;
    case 2: sincos_2pi(x, out[2 * i], out[2 * i + 1]); break;
    case 3: out[i] = hg_pdf(b[i], x); break;
    default: out[i] = hg_mu(b[i], x); break;
  }
}

int eval_functions(int32_t fn, int64_t n, const float* a, const float* b, float* out, int32_t on_device,
                   hipStream_t st) {
  if (fn < 0 || fn > 4 || n < 0 || n > (1ll << 30) || (n && (!a || !out || (fn >= 3 && !b))))
    return fail(TET_ERR_INVALID_ARG, "tet_eval_functions: bad arguments");
  if (n == 0) return TET_OK;
  const int64_t nout = fn == 2 ? 2 * n : n, nin = fn >= 3 ? 2 * n : n;
  const float *da = a, *db = b;
  float* dout = out;
  char* tmp = nullptr;
  if (!on_device) {
    tmp = (char*)dev_alloc((size_t)(nin + nout) * 4);
    if (!tmp) return fail(TET_ERR_OUT_OF_MEMORY, "tet_eval_functions: scratch");
    float* ta = (float*)tmp;
    TV_HIP(hipMemcpyAsync(ta, a, n * 4, hipMemcpyHostToDevice, st));
    if (fn >= 3) TV_HIP(hipMemcpyAsync(ta + n, b, n * 4, hipMemcpyHostToDevice, st));
    da = ta;
    db = ta + n;
    dout = ta + nin;
  }
  struct Free {
    void* p;
    ~Free() { if (p) dev_free(p); }
  } f_{tmp};
  hipLaunchKernelGGL(k_eval_functions, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)fn, n, da,
                     fn >= 3 ? db : nullptr, dout);
  TV_HIP(hipGetLastError());
  if (!on_device) TV_HIP(hipMemcpyAsync(out, dout, nout * 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

}  // namespace tv
