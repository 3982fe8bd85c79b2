// build.hip -- data-parallel construction of the adaptive, conforming
// tetrahedral grid (paper, "Grid Construction").
//
// The paper refines from its control cube by Maubach's longest-edge
// bisection and propagates every bisection to neighbours by a deterministic
// rule that keeps the grid conforming.  Here the same grid is reached by
// level-synchronous rounds:
//   mark:  a leaf splits if it is wanted (subdivision criteria) or if a mesh
//          vertex sits on the midpoint of one of its edges (a hanging vertex:
//          some neighbour across that edge has been bisected); the criteria
//          depend on the leaf alone, so they run once per leaf, over a dense
//          list of the leaves the previous round made;
//   scan:  exclusive scan of (1 + split) gives every leaf its new position;
//          children replace their parent in place, so depth-first order is
//          kept without sorting;
//   split: Maubach children are written and the new midpoint vertices are
//          inserted into a device hash set of mesh vertices.
// Every split made is necessary in any conforming refinement without wanted
// leaves, and the rounds stop at a conforming, want-free grid, so the result
// is the unique minimal one -- the grid the recursive propagation builds.
//
// Finalize: extinction / majorant per tet from the density pyramid, face
// orientation codes, and face neighbours found by locating a point just
// outside each face (face centroid pushed outward by a symbolic epsilon):
// exact integer descent from the root, then a binary search of the sorted
// depth-first keys.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace tv {

// ---------------------------------------------------------------- pyramid
__global__ void k_pyramid_level(const float* __restrict__ dens, const float* __restrict__ cmn,
                                const float* __restrict__ cmx, const double* __restrict__ csum, int32_t m,
                                float* __restrict__ mn, float* __restrict__ mx, double* __restrict__ sum) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)m * m * m;
  if (idx >= total) return;
  int64_t i = idx % m, j = (idx / m) % m, k = idx / ((int64_t)m * m);
  int64_t pm = 2 * (int64_t)m;
  float lo[8], hi[8];
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; q++) {
    int64_t c = (2 * i + (q & 1)) + pm * ((2 * j + ((q >> 1) & 1)) + pm * (2 * k + ((q >> 2) & 1)));
    if (dens) {
      float v = dens[c];
      lo[q] = v;
      hi[q] = v;
      s[q] = (double)v;
    } else {
      lo[q] = cmn[c];
      hi[q] = cmx[c];
      s[q] = csum[c];
    }
  }
  float a = lo[0], b = hi[0];
#pragma unroll
  for (int q = 1; q < 8; q++) {
    a = lo[q] < a ? lo[q] : a;
    b = hi[q] > b ? hi[q] : b;
  }
  mn[idx] = a;
  mx[idx] = b;
  sum[idx] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__global__ void k_check_density(const float* __restrict__ d, int64_t n, int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float v = d[i];
    if (!(v >= 0.0f) || isinf(v)) atomicOr(bad, 1);
  }
}

// Extra channels: value ranges (kind 0 temperature >= 0 and finite, 1
// albedo in [0, 1], 2 phase parameter g in (-1, 1)).
__global__ void k_check_channel(const float* __restrict__ d, int64_t n, int kind, int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float v = d[i];
    const bool ok = kind == 0 ? (v >= 0.0f && !isinf(v)) : (kind == 1 ? (v >= 0.0f && v <= 1.0f) : (v > -1.0f && v < 1.0f));
    if (!ok) atomicOr(bad, 1);
  }
}

// Statistics D(box) of the voxels overlapping the open lattice box (lo, hi):
// voxel range [lo / vs, ceil(hi / vs)) per axis, summarised at the coarsest
// pyramid level whose cells tile that range, cells combined in ascending
// z, y, x order.
__device__ inline void box_stats(const Pyramid& P, const int32_t lo[3], const int32_t hi[3], float& mn, float& mx,
                                 double& sum, double& cnt) {
  int sh = kLatBits - P.L;  // voxel size 2^sh lattice units
  int32_t r0[3], r1[3];
  int l = P.L;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    r0[a] = lo[a] >> sh;
    r1[a] = (hi[a] + (1 << sh) - 1) >> sh;
    if (r0[a] != 0) l = min(l, (int)__builtin_ctz((uint32_t)r0[a]));
    l = min(l, (int)__builtin_ctz((uint32_t)r1[a]));
  }
  int64_t m = (int64_t)P.n >> l;
  double s = 0.0;
  float a = 0.0f, b = 0.0f;
  bool first = true;
  int64_t cells = 0;
  for (int32_t k = r0[2] >> l; k < (r1[2] >> l); k++)
    for (int32_t j = r0[1] >> l; j < (r1[1] >> l); j++)
      for (int32_t i = r0[0] >> l; i < (r1[0] >> l); i++) {
        int64_t o = i + m * (j + m * (int64_t)k);
        float cmn, cmx;
        double cs;
        if (P.bmap && l < kBrickBits) {  // sparse levels 0..2: inside the cell's brick, zero without one
          const int sb = kBrickBits - l;
          const int32_t br = P.bmap[(i >> sb) + (int64_t)P.nb * ((j >> sb) + (int64_t)P.nb * (k >> sb))];
          if (br < 0) {
            cmn = cmx = 0.0f;
            cs = 0.0;
          } else {
            const int32_t mk = (1 << sb) - 1;
            const int64_t li = (int64_t)br * (1 << (3 * sb)) + ((i & mk) + ((j & mk) << sb) + ((k & mk) << (2 * sb)));
            if (l == 0) {
              cmn = cmx = P.bval[li];
              cs = (double)cmn;
            } else {
              cmn = P.bmn[l][li];
              cmx = P.bmx[l][li];
              cs = P.bsum[l][li];
            }
          }
        } else if (l == 0) {
          cmn = cmx = P.dens[o];
          cs = (double)cmn;
        } else {
          cmn = P.mn[l][o];
          cmx = P.mx[l][o];
          cs = P.sum[l][o];
        }
        if (first || cmn < a) a = cmn;
        if (first || cmx > b) b = cmx;
        first = false;
        s = s + cs;
        cells++;
      }
  mn = a;
  mx = b;
  sum = s;
  cnt = (double)cells * (double)(1ll << (3 * l));
}

__device__ inline void tet_box(const uint64_t v[4], int32_t lo[3], int32_t hi[3]) {
  int32_t x[4] = {vx(v[0]), vx(v[1]), vx(v[2]), vx(v[3])};
  int32_t y[4] = {vy(v[0]), vy(v[1]), vy(v[2]), vy(v[3])};
  int32_t z[4] = {vz(v[0]), vz(v[1]), vz(v[2]), vz(v[3])};
  lo[0] = min(min(x[0], x[1]), min(x[2], x[3]));
  hi[0] = max(max(x[0], x[1]), max(x[2], x[3]));
  lo[1] = min(min(y[0], y[1]), min(y[2], y[3]));
  hi[1] = max(max(y[0], y[1]), max(y[2], y[3]));
  lo[2] = min(min(z[0], z[1]), min(z[2], z[3]));
  hi[2] = max(max(z[0], z[1]), max(z[2], z[3]));
}

__device__ inline double dot3d(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

// Camera criterion: frustum test of the centroid with bounding radius l =
// longest edge, and projected size l k_px / z > target (all FP64).
__device__ inline bool want_camera(const CamCrit& cc, const uint64_t v[4], int depth) {
  int k = tag_of(depth);
  uint64_t vk = k == 1 ? v[1] : (k == 2 ? v[2] : v[3]);
  double w[3];
  int64_t sx = (int64_t)vx(v[0]) + vx(v[1]) + vx(v[2]) + vx(v[3]);
  int64_t sy = (int64_t)vy(v[0]) + vy(v[1]) + vy(v[2]) + vy(v[3]);
  int64_t sz = (int64_t)vz(v[0]) + vz(v[1]) + vz(v[2]) + vz(v[3]);
  w[0] = (double)sx * 0x1p-22 - cc.pos[0];
  w[1] = (double)sy * 0x1p-22 - cc.pos[1];
  w[2] = (double)sz * 0x1p-22 - cc.pos[2];
  int64_t ex = (int64_t)vx(vk) - vx(v[0]), ey = (int64_t)vy(vk) - vy(v[0]), ez = (int64_t)vz(vk) - vz(v[0]);
  int64_t l2i = ex * ex + ey * ey + ez * ez;
  double l2 = (double)l2i * 0x1p-40;
  double l = sqrt(l2);
  if (dot3d(cc.f, w) < -l) return false;
#pragma unroll
  for (int s = 0; s < 4; s++)
    if (dot3d(cc.side[s], w) < -l) return false;
  double z2 = dot3d(w, w);
  if (z2 <= l2) return true;
  return l2 * cc.kpx2 > cc.tgt2 * z2;
}

__device__ inline bool want(const Pyramid& P, const CamCrit& cc, const WantParams& wp, const uint64_t v[4],
                            uint64_t id) {
  int depth = id_depth(id);
  if (wp.mode == 1) return depth < wp.uniform_depth;
  if (wp.mode == 2) return depth < wp.max_depth && (int32_t)(mix64(id ^ wp.rand_seed) & 0xFFFF) < wp.rand_thresh;
  if (depth >= wp.max_depth) return false;
  int32_t lo[3], hi[3];
  tet_box(v, lo, hi);
  float mn, mx;
  double s, c;
  box_stats(P, lo, hi, mn, mx, s, c);
  double mean = s / c;
  if (!(mean > 0.0)) return false;
  if (!(((double)mx - (double)mn) > wp.tau * mean)) return false;
  return want_camera(cc, v, depth);
}

// Per-tet value of a channel: the mean over the voxels of the tet's box
// (the extinction's rule and summation order).
__global__ void k_channel_means(int64_t n, const uint64_t* __restrict__ verts, Pyramid P, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t v[4] = {verts[4 * t], verts[4 * t + 1], verts[4 * t + 2], verts[4 * t + 3]};
  int32_t lo[3], hi[3];
  tet_box(v, lo, hi);
  float mn, mx;
  double s, c;
  box_stats(P, lo, hi, mn, mx, s, c);
  out[t] = (float)(s / c);
}

// ---------------------------------------------------------------- vertex set
__device__ inline bool vset_has(const uint64_t* __restrict__ tab, uint64_t mask, uint64_t key) {
  uint64_t h = mix64(key) & mask;
  for (;;) {
    uint64_t e = tab[h];
    if (e == key) return true;
    if (e == kEmptyKey) return false;
    h = (h + 1) & mask;
  }
}

// Inserts key; true when it was not there before.
__device__ inline bool vset_add(uint64_t* tab, uint64_t mask, uint64_t key) {
  uint64_t h = mix64(key) & mask;
  for (;;) {
    unsigned long long prev = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)kEmptyKey,
                                        (unsigned long long)key);
    if (prev == kEmptyKey) return true;
    if (prev == key) return false;
    h = (h + 1) & mask;
  }
}

// One atomic per wave for a running count (called by every lane of the
// wave, in uniform control flow).
__device__ inline void count_new(bool added, uint32_t* count) {
  unsigned long long m = __ballot(added);
  if (m && __lane_id() == (int)__builtin_ctzll(m)) atomicAdd(count, (uint32_t)__popcll(m));
}

// The vertex count lives in kCountSlots words that the host sums: a block
// adds its total once, to the slot of its index, so the atomics of a large
// pass spread over kCountSlots addresses (on one address they serialise).
// Called by every thread of the block, in uniform control flow.
constexpr int kCountSlots = 16;

__device__ inline void block_count(bool x, uint32_t* slots) {
  __shared__ uint32_t s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const unsigned long long m = __ballot(x);
  if (m && __lane_id() == 0) atomicAdd(&s_n, (uint32_t)__popcll(m));
  __syncthreads();
  if (threadIdx.x == 0 && s_n) atomicAdd(&slots[blockIdx.x % kCountSlots], s_n);
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_vset_rehash(const uint64_t* __restrict__ old, int64_t ocap, uint64_t* tab, uint64_t mask,
                              uint32_t* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool added = i < ocap && old[i] != kEmptyKey && vset_add(tab, mask, old[i]);
  block_count(added, count);
}

// The vertices of n leaves (their 4 n packed vertices, with repeats).
__global__ void k_vset_seed(const uint64_t* __restrict__ verts, int64_t n, uint64_t* tab, uint64_t mask,
                            uint32_t* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool added = i < 4 * n && vset_add(tab, mask, verts[i]);
  block_count(added, count);
}

// ---------------------------------------------------------------- rounds
// Leaf flags: bit 0 = the want predicate was false (it depends on the tet
// alone, so it stays false); bit 1 = no mesh vertex sat on an edge midpoint
// at the leaf's last check.  A leaf with bit 1 can only have gained such a
// vertex from the last split pass, so it probes only the set of vertices
// that pass created (nset) instead of all of them.

// True when a vertex of `tab` sits on one of the tet's 6 edge midpoints;
// the first probes are issued together, collision chains followed only
// where the first slot holds another key.
__device__ inline bool hanging(const uint64_t v[4], const uint64_t* __restrict__ tab, uint64_t mask) {
  uint64_t key[6], h[6], e[6];
  bool on[6];
  int k = 0;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = a + 1; b < 4; b++, k++) {
      int32_t x = vx(v[a]) + vx(v[b]), y = vy(v[a]) + vy(v[b]), z = vz(v[a]) + vz(v[b]);
      on[k] = ((x | y | z) & 1) == 0;  // a midpoint on the lattice
      key[k] = pack_vertex(x >> 1, y >> 1, z >> 1);
      h[k] = mix64(key[k]) & mask;
    }
#pragma unroll
  for (k = 0; k < 6; k++) e[k] = on[k] ? tab[h[k]] : kEmptyKey;
  bool hit = false;
#pragma unroll
  for (k = 0; k < 6; k++) {
    if (!on[k] || hit) continue;
    if (e[k] == key[k]) hit = true;
    else if (e[k] != kEmptyKey) hit = vset_has(tab, mask, key[k]);
  }
  return hit;
}

// Cells of a 64^3 grid over the cube that received a vertex in the last
// split pass, one bit per cell, 0 = received (the map is cleared to all
// ones with the new-vertex set).  32 KB: it stays in the L1 caches.  An edge
// midpoint lies in the tet's bounding box, so a leaf whose box touches no
// marked cell cannot have gained a hanging vertex.
constexpr int kCellShift = kLatBits - 6;
constexpr int kCellWords = (64 * 64 * 64) / 32;
// followed by a coarse map, one bit per 8^3 cells (16 words, same sense)
constexpr int kCoarseWords = (8 * 8 * 8) / 32;
constexpr int kMapWords = kCellWords + kCoarseWords;

__device__ inline int cell_of(int32_t c) { return min(c >> kCellShift, 63); }

// Marks z's cell; with coarse, also its 8^3 region (tail rounds only: the
// coarse map has 16 words, so a bit already marked is not written again).
__device__ inline void cell_mark(uint32_t* cells, uint64_t z, bool coarse) {
  const int x = cell_of(vx(z)), y = cell_of(vy(z)), w = cell_of(vz(z));
  const int idx = (w * 64 + y) * 64 + x;
  atomicAnd(&cells[idx >> 5], ~(1u << (idx & 31)));
  if (coarse) {
    const int cidx = ((w >> 3) * 8 + (y >> 3)) * 8 + (x >> 3);
    const uint32_t cbit = 1u << (cidx & 31);
    if (__hip_atomic_load(&cells[kCellWords + (cidx >> 5)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & cbit)
      atomicAnd(&cells[kCellWords + (cidx >> 5)], ~cbit);
  }
}

// True when the box of v touches a marked cell (or spans more than 64 cells).
__device__ inline bool cells_touched(const uint32_t* __restrict__ cells, const uint64_t v[4]) {
  int32_t lo[3], hi[3];
  tet_box(v, lo, hi);
  const int x0 = cell_of(lo[0]), x1 = cell_of(hi[0]), y0 = cell_of(lo[1]), y1 = cell_of(hi[1]);
  const int z0 = cell_of(lo[2]), z1 = cell_of(hi[2]);
  if ((x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1) > 64) return true;
  for (int z = z0; z <= z1; z++)
    for (int y = y0; y <= y1; y++)
      for (int x = x0; x <= x1; x++) {
        const int idx = (z * 64 + y) * 64 + x;
        if (!((cells[idx >> 5] >> (idx & 31)) & 1u)) return true;
      }
  return false;
}

// Tail rounds: every leaf that splits is listed.  The list positions come
// from the running split count (one atomic per wave); list0 is its value at
// the start of the round.
__device__ inline void list_split(bool split, uint32_t i, uint32_t* splitc, uint32_t list0, uint32_t* slist) {
  const unsigned long long m = __ballot(split);
  if (!m) return;
  const int lane = __lane_id(), leader = (int)__builtin_ctzll(m);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(splitc, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (split) slist[base - list0 + (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull))] = i;
}

// Tail rounds keep, per chunk of 256 leaves of the main part, a box of
// cells holding every leaf of the chunk: min x, y, z at words 0..2 and max
// at 4..6 of 8.  Child 0 stays inside its parent's box, so the boxes stay
// valid while the tail rounds split leaves in place.
constexpr int kChunk = 256;

__device__ inline void cell_box(const uint64_t v[4], uint32_t c[6]) {
  int32_t lo[3], hi[3];
  tet_box(v, lo, hi);
#pragma unroll
  for (int a = 0; a < 3; a++) {
    c[a] = (uint32_t)cell_of(lo[a]);
    c[3 + a] = (uint32_t)cell_of(hi[a]);
  }
}

// Boxes of chunks [c0, c1) over the leaves below n (empty past n).
__global__ void k_chunk_boxes(int64_t n, int64_t c0, int64_t c1, const uint64_t* __restrict__ verts,
                              uint32_t* __restrict__ box) {
  const int64_t c = c0 + blockIdx.x;
  const int64_t i = c * kChunk + threadIdx.x;
  uint32_t b[6] = {63, 63, 63, 0, 0, 0};
  if (i < n) {
    uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]};
    cell_box(v, b);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      b[a] = min(b[a], (uint32_t)__shfl_xor(b[a], off, 64));
      b[3 + a] = max(b[3 + a], (uint32_t)__shfl_xor(b[3 + a], off, 64));
    }
  __shared__ uint32_t sb[kChunk / 64][6];
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0)
    for (int a = 0; a < 6; a++) sb[w][a] = b[a];
  __syncthreads();
  if (threadIdx.x < 8) {
    uint32_t r = threadIdx.x < 3 ? 63u : 0u;
    for (int k = 0; k < kChunk / 64; k++) {
      if (threadIdx.x < 3) r = min(r, sb[k][threadIdx.x]);
      else if (threadIdx.x >= 4 && threadIdx.x < 7) r = max(r, sb[k][threadIdx.x - 1]);
    }
    if (c < c1) box[8 * c + threadIdx.x] = r;
  }
}

// True when the chunk's box may hold a marked cell.
__device__ inline bool chunk_touched(const uint32_t* __restrict__ cells, const uint32_t* __restrict__ box,
                                     int64_t c) {
  const uint32_t x0 = box[8 * c], y0 = box[8 * c + 1], z0 = box[8 * c + 2];
  const uint32_t x1 = box[8 * c + 4], y1 = box[8 * c + 5], z1 = box[8 * c + 6];
  if (x0 > x1) return false;  // empty
  if ((x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1) > 64) return true;
  for (uint32_t z = z0; z <= z1; z++)
    for (uint32_t y = y0; y <= y1; y++)
      for (uint32_t x = x0; x <= x1; x++) {
        const uint32_t idx = (z * 64 + y) * 64 + x;
        if (!((cells[idx >> 5] >> (idx & 31)) & 1u)) return true;
      }
  return false;
}

// Leaves whose want predicate is settled: split only when forced.
__global__ void k_mark(int64_t n, const uint64_t* __restrict__ verts, uint8_t* __restrict__ flags,
                       uint32_t* __restrict__ cnt, const uint64_t* __restrict__ vset, uint64_t vmask,
                       const uint64_t* __restrict__ nset, uint64_t nmask, const uint32_t* __restrict__ cells,
                       uint32_t* splitc, uint32_t list0, uint32_t* __restrict__ slist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool split = false;
  if (i < n) {
    const uint8_t fl = flags[i];
    if (fl & 1) {  // new leaves (flag 0) are k_want's
      uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]};
      // checked leaves: the last pass's new vertices (after a dense pass,
      // nset is the whole vertex set and there is no cell map)
      if (fl & 2) split = (!cells || cells_touched(cells, v)) && hanging(v, nset, nmask);
      else split = hanging(v, vset, vmask);
      if (!split && !(fl & 2)) flags[i] = fl | 2;
      if (!slist) cnt[i] = split ? 2u : 1u;
    }
  }
  if (slist) list_split(split, (uint32_t)i, splitc, list0, slist);
}

// Tail rounds: k_mark over chunks, kTailChunks per block, with the cell
// map staged in LDS.  A chunk of the main part whose box holds no marked
// cell is skipped whole: its leaves are all checked (flag bit 1; the tail
// starts after a compacting round, which checks every leaf), so none can
// split.  Chunks holding appended leaves are always read.  Each half-wave
// tests one chunk's box, a cell per lane (boxes of more than 64 cells count
// as touched).
constexpr int kTailChunks = 8;

__device__ inline bool cell_marked(const uint32_t* m, uint32_t x, uint32_t y, uint32_t z) {
  const uint32_t idx = (z * 64 + y) * 64 + x;
  return !((m[idx >> 5] >> (idx & 31)) & 1u);
}

__global__ __launch_bounds__(kChunk) void k_mark_tail(int64_t n, int64_t nmain, const uint64_t* __restrict__ verts,
                                                      uint8_t* __restrict__ flags, const uint64_t* __restrict__ vset,
                                                      uint64_t vmask, const uint64_t* __restrict__ nset,
                                                      uint64_t nmask, const uint32_t* __restrict__ cells,
                                                      const uint32_t* __restrict__ box, uint32_t* splitc,
                                                      uint32_t list0, uint32_t* __restrict__ slist, int coarse) {
  static_assert(kChunk == 256 && kTailChunks == 8, "two chunks per wave of the block");
  __shared__ uint4 smap4[kCellWords / 4];
  __shared__ int stouch[kTailChunks];
  // coarse test first (when the last split was a tail round's, which keeps
  // the coarse map): a block none of whose chunks meets a marked 8^3 region
  // stages nothing
  if (coarse) {
    const int lane = __lane_id(), k = 2 * (threadIdx.x >> 6) + (lane >> 5), j = lane & 31;
    const int64_t c = (int64_t)blockIdx.x * kTailChunks + k;
    bool hit = false;
    if (c * kChunk < n) {
      if (c >= nmain / kChunk) {
        hit = true;
      } else {
        const uint32_t x0 = box[8 * c] >> 3, y0 = box[8 * c + 1] >> 3, z0 = box[8 * c + 2] >> 3;
        const uint32_t nx = (box[8 * c + 4] >> 3) - x0 + 1, ny = (box[8 * c + 5] >> 3) - y0 + 1;
        const uint32_t nz = (box[8 * c + 6] >> 3) - z0 + 1;
        for (uint32_t q = j; q < nx * ny * nz; q += 32) {
          const uint32_t cidx = ((z0 + q / (nx * ny)) * 8 + (y0 + (q / nx) % ny)) * 8 + (x0 + q % nx);
          hit = hit || !((cells[kCellWords + (cidx >> 5)] >> (cidx & 31)) & 1u);
        }
      }
    }
    if (!__syncthreads_or(hit)) return;
  }
  const uint4* c4 = reinterpret_cast<const uint4*>(cells);
  for (int w = threadIdx.x; w < kCellWords / 4; w += kChunk) smap4[w] = c4[w];
  __syncthreads();
  const uint32_t* smap = reinterpret_cast<const uint32_t*>(smap4);
  {
    const int lane = __lane_id(), k = 2 * (threadIdx.x >> 6) + (lane >> 5), j = lane & 31;
    const int64_t c = (int64_t)blockIdx.x * kTailChunks + k;
    bool hit = false, all = false;
    if (c * kChunk < n) {
      if (c >= nmain / kChunk) {
        all = true;
      } else {
        const uint32_t x0 = box[8 * c], y0 = box[8 * c + 1], z0 = box[8 * c + 2];
        const uint32_t nx = box[8 * c + 4] - x0 + 1, ny = box[8 * c + 5] - y0 + 1, nz = box[8 * c + 6] - z0 + 1;
        const uint32_t cnt = nx * ny * nz;
        if (cnt > 64) all = true;
        for (uint32_t q = j; q < cnt && q < 64; q += 32)
          hit = hit || cell_marked(smap, x0 + q % nx, y0 + (q / nx) % ny, z0 + q / (nx * ny));
      }
    }
    const unsigned long long m = __ballot(hit || all);
    if (j == 0) stouch[k] = ((m >> (lane & 32)) & 0xFFFFFFFFull) != 0;
  }
  __syncthreads();
  for (int k = 0; k < kTailChunks; k++) {
    if (!stouch[k]) continue;
    const int64_t i = ((int64_t)blockIdx.x * kTailChunks + k) * kChunk + threadIdx.x;
    bool split = false;
    if (i < n) {
      const uint8_t fl = flags[i];
      if (fl & 1) {
        uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]};
        if (fl & 2) {
          uint32_t cb[6];
          cell_box(v, cb);
          bool t = (cb[3] - cb[0] + 1) * (cb[4] - cb[1] + 1) * (cb[5] - cb[2] + 1) > 64;
          for (uint32_t z = cb[2]; z <= cb[5] && !t; z++)
            for (uint32_t y = cb[1]; y <= cb[4] && !t; y++)
              for (uint32_t x = cb[0]; x <= cb[3] && !t; x++) t = cell_marked(smap, x, y, z);
          split = t && hanging(v, nset, nmask);
        } else {
          split = hanging(v, vset, vmask);
          if (!split) flags[i] = fl | 2;
        }
      }
    }
    list_split(split, (uint32_t)i, splitc, list0, slist);
  }
}

// The leaves made by the last split pass (a dense list, so the want
// predicate's FP64 work runs on full waves): wanted, or forced.
__global__ void k_want(int64_t m, const uint32_t* __restrict__ work, const uint64_t* __restrict__ ids,
                       const uint64_t* __restrict__ verts, uint8_t* __restrict__ flags, uint32_t* __restrict__ cnt,
                       Pyramid P, CamCrit cc, WantParams wp, const uint64_t* __restrict__ vset, uint64_t vmask,
                       uint32_t* splitc, uint32_t list0, uint32_t* __restrict__ slist) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool split = false;
  uint32_t i = 0;
  if (j < m) {
    i = work[j];
    uint64_t v[4] = {verts[4 * (size_t)i], verts[4 * (size_t)i + 1], verts[4 * (size_t)i + 2],
                     verts[4 * (size_t)i + 3]};
    split = want(P, cc, wp, v, ids[i]);
    uint8_t nf = 0;
    if (!split) {
      nf = 1;
      split = hanging(v, vset, vmask);
      if (!split) nf = 3;
    }
    flags[i] = nf;
    if (!slist) cnt[i] = split ? 2u : 1u;
  }
  if (slist) list_split(split, i, splitc, list0, slist);
}

// Maubach children of the tet (id, v): the first child replaces vertex x_k
// (k = tag) by the midpoint z of (x0, x_k), the second is (x1..x_k, z,
// x_{k+1}..x3).  Returns z.
__device__ inline uint64_t children(uint64_t id, const uint64_t v[4], uint64_t a[4], uint64_t b[4]) {
  uint64_t z;
  switch (tag_of(id_depth(id))) {
    case 1:
      z = vmid(v[0], v[1]);
      a[0] = v[0]; a[1] = z; a[2] = v[2]; a[3] = v[3];
      b[0] = v[1]; b[1] = z; b[2] = v[2]; b[3] = v[3];
      break;
    case 2:
      z = vmid(v[0], v[2]);
      a[0] = v[0]; a[1] = v[1]; a[2] = z; a[3] = v[3];
      b[0] = v[1]; b[1] = v[2]; b[2] = z; b[3] = v[3];
      break;
    default:
      z = vmid(v[0], v[3]);
      a[0] = v[0]; a[1] = v[1]; a[2] = v[2]; a[3] = z;
      b[0] = v[1]; b[1] = v[2]; b[2] = v[3]; b[3] = z;
      break;
  }
  return z;
}

// Want bits of a leaf's ancestor chain (bit d: the ancestor at depth d was
// split because the want predicate held, not only to keep the grid
// conforming).  A split leaf passes its chain on with its own bit: flag bit 0
// set means its predicate was false, so a conformity split.
__device__ inline uint64_t child_chain(uint64_t chain, uint8_t flag, uint64_t id) {
  return chain | ((flag & 1) ? 0ull : (1ull << id_depth(id)));
}

// Copies leaf i to position o, or writes its two children there and adds
// the new vertex to the vertex set (and to the new-vertex set when given);
// true when the vertex is new.
__device__ inline bool split_one(int64_t i, int64_t o, bool split, const uint64_t* ids, const uint64_t* verts,
                                 const uint8_t* flags, const uint64_t* chain, uint64_t* nids, uint64_t* nverts,
                                 uint8_t* nflags, uint64_t* nchain, uint64_t* vset, uint64_t vmask, uint64_t* nset,
                                 uint64_t nmask, uint32_t* cells, uint32_t* work) {
  uint64_t id = ids[i];
  uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]};
  if (!split) {
    nids[o] = id;
    nflags[o] = flags[i];
    nchain[o] = chain[i];
#pragma unroll
    for (int j = 0; j < 4; j++) nverts[4 * o + j] = v[j];
    return false;
  }
  uint64_t a[4], b[4];
  const uint64_t z = children(id, v, a, b);
  const uint64_t ch = child_chain(chain[i], flags[i], id);
  nids[o] = 2 * id;
  nids[o + 1] = 2 * id + 1;
  nflags[o] = 0;
  nflags[o + 1] = 0;
  nchain[o] = ch;
  nchain[o + 1] = ch;
  const int64_t r = o - i;  // splits before this leaf
  work[2 * r] = (uint32_t)o;
  work[2 * r + 1] = (uint32_t)(o + 1);
#pragma unroll
  for (int j = 0; j < 4; j++) {
    nverts[4 * o + j] = a[j];
    nverts[4 * (o + 1) + j] = b[j];
  }
  bool added = vset_add(vset, vmask, z);
  if (nset && added) {  // only vertices new to the mesh can hang on a checked leaf
    vset_add(nset, nmask, z);
    cell_mark(cells, z, false);
  }
  return added;
}

__global__ void k_split(int64_t n, const uint64_t* __restrict__ ids, const uint64_t* __restrict__ verts,
                        const uint8_t* __restrict__ flags, const uint64_t* __restrict__ chain,
                        const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ offs,
                        uint64_t* __restrict__ nids, uint64_t* __restrict__ nverts, uint8_t* __restrict__ nflags,
                        uint64_t* __restrict__ nchain, uint64_t* vset, uint64_t vmask, uint32_t* vcount,
                        uint64_t* nset, uint64_t nmask, uint32_t* cells, uint32_t* __restrict__ work) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool added = false;
  if (i < n)
    added = split_one(i, offs[i], cnt[i] != 1u, ids, verts, flags, chain, nids, nverts, nflags, nchain, vset, vmask,
                      nset, nmask, cells, work);
  block_count(added, vcount);
}


// Tail rounds, where few leaves split: no compaction.  Child 0 replaces its
// parent in place (its depth-first key is the parent's, so the leaves below
// nmain stay in key order), child 1 of the s-th listed leaf goes to n + s,
// and anc names the leaf below nmain it descends from.  The list is in no
// particular order, so neither are the appended leaves until k_merge.
__global__ void k_split_append(int64_t count, const uint32_t* __restrict__ slist, int64_t n, int64_t nmain,
                               uint64_t* __restrict__ ids, uint64_t* __restrict__ verts,
                               uint8_t* __restrict__ flags, uint64_t* __restrict__ chain,
                               uint32_t* __restrict__ anc, uint64_t* vset,
                               uint64_t vmask, uint32_t* vcount, uint64_t* nset, uint64_t nmask, uint32_t* cells,
                               uint32_t* __restrict__ work) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool added = false;
  if (s < count) {
    const int64_t i = slist[s], o = n + s;
    const uint64_t id = ids[i];
    uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]}, a[4], b[4];
    const uint64_t z = children(id, v, a, b);
    const uint64_t ch = child_chain(chain[i], flags[i], id);
    ids[i] = 2 * id;
    ids[o] = 2 * id + 1;
    flags[i] = 0;
    flags[o] = 0;
    chain[i] = ch;
    chain[o] = ch;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      verts[4 * i + j] = a[j];
      verts[4 * o + j] = b[j];
    }
    anc[o - nmain] = i < nmain ? (uint32_t)i : anc[i - nmain];
    work[2 * s] = (uint32_t)i;
    work[2 * s + 1] = (uint32_t)o;
    added = vset_add(vset, vmask, z);
    if (added) {
      vset_add(nset, nmask, z);
      cell_mark(cells, z, true);
    }
  }
  block_count(added, vcount);
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Merge of the appended leaves: g[i] = 1 + the number of appended leaves
// descending from leaf i (g starts at 1).
__global__ void k_group_count(int64_t m, const uint32_t* __restrict__ anc, uint32_t* g) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) atomicAdd(&g[anc[j]], 1u);
}

// With pos = exclusive scan of g, leaf i goes to pos[i] and its appended
// descendants fill pos[i] + 1 .. pos[i] + g[i] - 1; slots lists them there
// in arrival order (fill starts at 0).
__global__ void k_group_slots(int64_t m, const uint32_t* __restrict__ anc, const uint32_t* __restrict__ pos,
                              uint32_t* fill, uint32_t* __restrict__ slots) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint32_t i = anc[j];
  slots[pos[i] + 1 + atomicAdd(&fill[i], 1u)] = (uint32_t)j;
}

__device__ inline uint64_t dfs_key(uint64_t id) { return id << (60 - id_depth(id)); }

// Writes the leaves in depth-first order: leaf i < nmain at pos[i], then its
// appended descendants ranked by key (they are leaves of one subtree, so
// their keys are distinct).
__global__ void k_merge(int64_t nmain, int64_t m, int64_t total, const uint64_t* __restrict__ ids,
                        const uint64_t* __restrict__ verts, const uint64_t* __restrict__ chain,
                        const uint32_t* __restrict__ anc, const uint32_t* __restrict__ pos,
                        const uint32_t* __restrict__ slots, uint64_t* __restrict__ out_ids,
                        uint64_t* __restrict__ out_verts, uint64_t* __restrict__ out_chain) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nmain + m) return;
  int64_t o;
  if (t < nmain) {
    o = pos[t];
  } else {
    const int64_t j = t - nmain;
    const uint32_t i = anc[j];
    const int64_t first = (int64_t)pos[i] + 1, end = i + 1 < nmain ? (int64_t)pos[i + 1] : total;
    const uint64_t key = dfs_key(ids[t]);
    int64_t r = 0;
    for (int64_t k = first; k < end; k++) r += dfs_key(ids[nmain + slots[k]]) < key;
    o = first + r;
  }
  out_ids[o] = ids[t];
  out_chain[o] = chain[t];
#pragma unroll
  for (int q = 0; q < 4; q++) out_verts[4 * o + q] = verts[4 * t + q];
}

// ---------------------------------------------------------------- scan
// Exclusive scan of n uint32 values, 1024 per block (256 threads x 4).
constexpr int kScanThreads = 256, kScanItems = 4, kScanBlock = kScanThreads * kScanItems;

__device__ inline uint32_t block_exclusive(uint32_t x, uint32_t* wsum, uint32_t* total) {
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < kScanThreads / 64; w++) {
    if (w < wid) pre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  if (total) *total = tot;
  return pre + inc - x;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t ws[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; q++)
    if (base + q < n) s += in[base + q];
  uint32_t tot;
  block_exclusive(s, ws, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_blocks(uint32_t* bsum, int64_t nb, uint32_t* total) {
  __shared__ uint32_t ws[kScanThreads / 64];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    int64_t i = base + threadIdx.x;
    uint32_t x = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive(x, ws, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_apply(const uint32_t* __restrict__ in, int64_t n, const uint32_t* __restrict__ bsum,
                             uint32_t* __restrict__ out) {
  __shared__ uint32_t ws[kScanThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; q++) {
    v[q] = base + q < n ? in[base + q] : 0u;
    s += v[q];
  }
  uint32_t ex = block_exclusive(s, ws, nullptr) + bsum[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItems; q++) {
    if (base + q < n) out[base + q] = ex;
    ex += v[q];
  }
}

// ---------------------------------------------------------------- seed from a previous grid
// A previous grid's tree seeds the rounds of a new build.  A node of that
// tree that satisfies the (new) want predicate, as all its ancestors do, is
// split in the new grid as well: the rounds from the roots split every
// wanted leaf, so such a node becomes a leaf at some round and is then split.
// The seed -- the previous tree cut at the first node of each branch that is
// not wanted, or at the previous leaf -- is therefore a stage that the rounds
// from the roots pass through, and the rounds continued from it end at the
// same grid, which does not depend on the order of the splits.  Leaves the
// new criteria no longer want are merged away by not being seeded; the
// splits that conformity forced are found again by the rounds.
//
// Node a of the previous tree is owned by the first leaf of its subtree in
// depth-first order: leaf p owns itself and its ancestors below its deepest
// common ancestor with leaf p - 1.  Each leaf evaluates the predicate of the
// nodes it owns (bit d for the node at depth d), and an inclusive scan of
// M_p = (M_{p-1} & keep_p) | bits_p gives each leaf the bits of its whole
// ancestor chain and itself (keep_p: the depths it does not own).
//
// The previous grid keeps the same bits from its own build (its chain: the
// predicate of every ancestor; a leaf's own predicate was false).  When the
// new bits equal them for every leaf, the predicate takes the same value on
// every node of the previous tree, so a build from the roots under the new
// criteria makes exactly the same splits: the grid stands as it is.

// Lattice vertices of root r (the Kuhn tet of axis order (a, b, the third)).
__device__ inline void root_vertices(int r, uint64_t v[4]) {
  const int a = r >> 1;
  const int b = a == 0 ? ((r & 1) ? 2 : 1) : (a == 1 ? ((r & 1) ? 2 : 0) : ((r & 1) ? 1 : 0));
  int32_t c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
  c1[a] = kLatS;
  c2[a] = kLatS;
  c2[b] = kLatS;
  v[0] = pack_vertex(0, 0, 0);
  v[1] = pack_vertex(c1[0], c1[1], c1[2]);
  v[2] = pack_vertex(c2[0], c2[1], c2[2]);
  v[3] = pack_vertex(kLatS, kLatS, kLatS);
}

// Vertices of the depth-d ancestor of the tet with heap id h (depth D >= d),
// by bisecting down from its root.
__device__ inline void ancestor_vertices(uint64_t h, int D, int d, uint64_t v[4]) {
  root_vertices((int)(h >> D) - 8, v);
  for (int e = 0; e < d; e++) {
    uint64_t c0[4], c1[4];
    children(h >> (D - e), v, c0, c1);
    const bool right = (h >> (D - e - 1)) & 1;
#pragma unroll
    for (int j = 0; j < 4; j++) v[j] = right ? c1[j] : c0[j];
  }
}

// Depth of the deepest common ancestor of two distinct leaves (-1: roots differ).
__device__ inline int common_depth(uint64_t a, uint64_t b) {
  const int da = id_depth(a), db = id_depth(b), m = min(da, db);
  const uint64_t x = (a >> (da - m)) ^ (b >> (db - m));
  if (!x) return m;
  return max(m - (64 - (int)__builtin_clzll(x)), -1);
}

__global__ void k_seed_chain(int64_t n, const uint64_t* __restrict__ ids, Pyramid P, CamCrit cc, WantParams wp,
                             uint64_t* __restrict__ keep, uint64_t* __restrict__ bits) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t h = ids[p];
  const int D = id_depth(h);
  const int c = p ? common_depth(ids[p - 1], h) : -1;
  uint64_t v[4];
  root_vertices((int)(h >> D) - 8, v);
  uint64_t b = 0;
  for (int d = 0; d <= D; d++) {
    const uint64_t a = h >> (D - d);
    if (d > c && want(P, cc, wp, v, a)) b |= 1ull << d;
    if (d == D) break;
    uint64_t c0[4], c1[4];
    children(a, v, c0, c1);
    const bool right = (h >> (D - d - 1)) & 1;
#pragma unroll
    for (int j = 0; j < 4; j++) v[j] = right ? c1[j] : c0[j];
  }
  keep[p] = c >= 0 ? (~0ull >> (63 - c)) : 0ull;
  bits[p] = b;
}

// Transform M -> (M & k) | b of the chain scan; compose(x, y) applies x, then y.
struct ChainT {
  uint64_t k, b;
};
__device__ inline ChainT chain_compose(ChainT x, ChainT y) { return {x.k & y.k, (x.b & y.k) | y.b}; }

// Exclusive scan of one transform per thread over the block (kScanThreads);
// *total receives the block's whole composition.
__device__ inline ChainT block_chain_exclusive(ChainT x, ChainT* ws, ChainT* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  ChainT inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const ChainT y = {__shfl_up(inc.k, o, 64), __shfl_up(inc.b, o, 64)};
    if (lane >= o) inc = chain_compose(y, inc);
  }
  ChainT ex = {__shfl_up(inc.k, 1, 64), __shfl_up(inc.b, 1, 64)};
  if (lane == 0) ex = {~0ull, 0ull};
  if (lane == 63) ws[wid] = inc;
  __syncthreads();
  ChainT pre = {~0ull, 0ull}, tot = {~0ull, 0ull};
  for (int w = 0; w < kScanThreads / 64; w++) {
    if (w < wid) pre = chain_compose(pre, ws[w]);
    tot = chain_compose(tot, ws[w]);
  }
  __syncthreads();
  if (total) *total = tot;
  return chain_compose(pre, ex);
}

__device__ inline ChainT chain_items(const uint64_t* keep, const uint64_t* bits, int64_t base, int64_t n) {
  ChainT t = {~0ull, 0ull};
#pragma unroll
  for (int q = 0; q < kScanItems; q++)
    if (base + q < n) t = chain_compose(t, ChainT{keep[base + q], bits[base + q]});
  return t;
}

__global__ void k_chain_reduce(const uint64_t* __restrict__ keep, const uint64_t* __restrict__ bits, int64_t n,
                               ChainT* __restrict__ bagg) {
  __shared__ ChainT ws[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  ChainT tot;
  block_chain_exclusive(chain_items(keep, bits, base, n), ws, &tot);
  if (threadIdx.x == 0) bagg[blockIdx.x] = tot;
}

// One block: the chain bits entering each block, in place of its aggregate.
__global__ void k_chain_blocks(ChainT* bagg, int64_t nb) {
  __shared__ ChainT ws[kScanThreads / 64];
  ChainT carry = {~0ull, 0ull};
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const ChainT x = i < nb ? bagg[i] : ChainT{~0ull, 0ull};
    ChainT tot;
    const ChainT ex = block_chain_exclusive(x, ws, &tot);
    if (i < nb) bagg[i] = ChainT{0ull, chain_compose(carry, ex).b};  // applied to M = 0 before the first leaf
    carry = chain_compose(carry, tot);
  }
}

// M of every leaf, written over bits.
__global__ void k_chain_apply(const uint64_t* __restrict__ keep, uint64_t* __restrict__ bits, int64_t n,
                              const ChainT* __restrict__ bagg) {
  __shared__ ChainT ws[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint64_t k[kScanItems], b[kScanItems];
#pragma unroll
  for (int q = 0; q < kScanItems; q++) {
    k[q] = base + q < n ? keep[base + q] : ~0ull;
    b[q] = base + q < n ? bits[base + q] : 0ull;
  }
  ChainT t = {~0ull, 0ull};
#pragma unroll
  for (int q = 0; q < kScanItems; q++) t = chain_compose(t, ChainT{k[q], b[q]});
  const ChainT ex = block_chain_exclusive(t, ws, nullptr);
  uint64_t m = (bagg[blockIdx.x].b & ex.k) | ex.b;
#pragma unroll
  for (int q = 0; q < kScanItems; q++) {
    m = (m & k[q]) | b[q];
    if (base + q < n) bits[base + q] = m;
  }
}

// Seed node of leaf h with chain bits m: its ancestor at the first depth
// whose node is not wanted, or h itself; *wanted when the whole chain,
// h included, is wanted.
__device__ inline uint64_t seed_node(uint64_t h, uint64_t m, int* depth, bool* wanted) {
  const int D = id_depth(h);
  const int f = (int)__builtin_ctzll(~m);  // m has no bit above depth 56
  *wanted = f > D;
  *depth = min(f, D);
  return h >> (D - *depth);
}

__global__ void k_seed_first(int64_t n, const uint64_t* __restrict__ ids, const uint64_t* __restrict__ chain,
                             uint32_t* __restrict__ first) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int d;
  bool w;
  const uint64_t s = seed_node(ids[p], chain[p], &d, &w);
  first[p] = (p == 0 || seed_node(ids[p - 1], chain[p - 1], &d, &w) != s) ? 1u : 0u;
}

// Extinction and majorant of every tet of a grid whose tree stays, for the
// volume and scale of a new build (k_records' rule; the rest of the records
// depends on the tree alone).
__global__ void k_refresh_medium(int64_t n, const uint64_t* __restrict__ verts, Pyramid P, float scale,
                                 int majorant_mode, TetRec* __restrict__ rec, TetRec32* __restrict__ rec32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t pv[4] = {verts[4 * t], verts[4 * t + 1], verts[4 * t + 2], verts[4 * t + 3]};
  int32_t lo[3], hi[3];
  tet_box(pv, lo, hi);
  float mn, mx;
  double sm, c;
  box_stats(P, lo, hi, mn, mx, sm, c);
  const float sigma = (float)((double)scale * (sm / c));
  const float majorant = majorant_mode == 1 ? (float)((double)scale * (double)mx) : sigma;
  rec[t].sigma = sigma;
  rec[t].majorant = majorant;
  if (rec32) rec32[t].w[3] = __float_as_uint(sigma);
}

// Leaves whose chain bits differ from the previous grid's (one atomic per wave).
__global__ void k_chain_diff(int64_t n, const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                             uint32_t* count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool d = p < n && a[p] != b[p];
  count_new(d, count);
}

// Adds x over the block to slots[blockIdx.x % kCountSlots] (every thread of
// the block calls it, in uniform control flow).
__device__ inline void block_add(uint32_t x, uint32_t* slots) {
  __shared__ uint32_t s_n;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  if (x) atomicAdd(&s_n, x);
  __syncthreads();
  if (threadIdx.x == 0 && s_n) atomicAdd(&slots[blockIdx.x % kCountSlots], s_n);
}

// The seed's leaves in depth-first order, with their chains and the flags of
// the rounds (0: wanted, listed for k_want; 1: not wanted, checked by k_mark
// against the whole vertex set).  The seed's vertices are the cube's corners
// and the midpoints of its split nodes; the first leaf of each seed node's
// run owns the split nodes above it that the previous tree's ownership gives
// it (depths c < d < m), and adds their midpoints to the vertex set.
__global__ void k_seed_write(int64_t n, const uint64_t* __restrict__ ids, const uint64_t* __restrict__ chain,
                             const uint32_t* __restrict__ first, const uint32_t* __restrict__ pos,
                             uint64_t* __restrict__ sids, uint64_t* __restrict__ sverts, uint8_t* __restrict__ sflags,
                             uint64_t* __restrict__ schain, uint32_t* __restrict__ work, uint32_t* count,
                             uint64_t* vset, uint64_t vmask, uint32_t* vcount) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool listed = false;
  uint32_t o = 0, added = 0;
  if (p == 0) {  // the corners
    for (int q = 0; q < 8; q++)
      added += vset_add(vset, vmask, pack_vertex((q & 1) ? kLatS : 0, (q & 2) ? kLatS : 0, (q & 4) ? kLatS : 0));
  }
  if (p < n && first[p]) {
    const uint64_t h = ids[p];
    const int D = id_depth(h);
    const int c = p ? common_depth(ids[p - 1], h) : -1;
    int m;
    bool w;
    const uint64_t sd = seed_node(h, chain[p], &m, &w);
    uint64_t v[4];
    root_vertices((int)(h >> D) - 8, v);
    for (int d = 0; d < m; d++) {
      uint64_t c0[4], c1[4];
      const uint64_t z = children(h >> (D - d), v, c0, c1);
      if (d > c) added += vset_add(vset, vmask, z);
      const bool right = (h >> (D - d - 1)) & 1;
#pragma unroll
      for (int j = 0; j < 4; j++) v[j] = right ? c1[j] : c0[j];
    }
    o = pos[p];
    sids[o] = sd;
#pragma unroll
    for (int j = 0; j < 4; j++) sverts[4 * (size_t)o + j] = v[j];
    sflags[o] = w ? 0 : 1;
    schain[o] = m ? (~0ull >> (64 - m)) : 0ull;  // every ancestor of a seed node is wanted
    listed = w;
  }
  block_add(added, vcount);
  const unsigned long long mk = __ballot(listed);
  if (mk) {
    const int lane = __lane_id(), leader = (int)__builtin_ctzll(mk);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mk));
    base = __shfl(base, leader, 64);
    if (listed) work[base + (uint32_t)__popcll(mk & (lane ? (~0ull >> (64 - lane)) : 0ull))] = o;
  }
}

// ---------------------------------------------------------------- small grids
// While the grid is small a round holds too little work to hide the cost of
// its launches and of the host reading the leaf count back, so the first
// rounds run in one cooperative launch (every block resident): each block
// owns a contiguous chunk of the leaves, and a round is mark, grid barrier,
// offsets from the per-block counts and split, grid barrier.  The kernel
// stops when the grid is conforming and want-free, or once it holds more
// than cap / 2 leaves (the next round could then exceed cap).  Marking
// probes the whole vertex set (flag bit 1 is never set here), and the last
// split leaves the list of its new leaves for the rounds that follow.
constexpr uint32_t kBarrierSpins = 1u << 24;  // about a second of s_sleep per barrier
constexpr int64_t kSmallCap = 1 << 21;         // leaves the cooperative rounds may reach
constexpr int64_t kAppendRatio = 16;           // tail rounds: fewer than leaves / 16 splits

struct SmallRounds {
  uint64_t* ids[2];
  uint64_t* verts[2];
  uint8_t* flags[2];
  uint64_t* chain[2];
  uint32_t* cnt;    // per leaf: 1 or 2
  uint32_t* bsum;   // per block: sum of cnt over its chunk
  uint32_t* work;   // new leaves of the last split
  uint64_t* vset;
  uint64_t vmask;
  uint32_t* vcount;
  uint32_t* state;  // out: [0] leaves, [1] rounds, [2] splits of the last round, [3] converged;
                    // [4] barrier arrivals (zero at launch), [5] nonzero: a barrier timed out
  int64_t cur0, cap;
};

// Grid barrier number k (1, 2, ...): every block adds one arrival, then waits
// until k * gridDim.x arrivals are in.  The wait is bounded; on time-out the
// error word is set and every block leaves the kernel at its next check.
__device__ inline bool grid_barrier(uint32_t* arrivals, uint32_t* err, uint32_t k, int* s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(arrivals, 1u);
    const uint32_t target = k * gridDim.x;
    int ok = 1;
    // relaxed polling (an acquiring load would invalidate this XCD's L2 on
    // every poll, under the blocks still working); one fence after the wait
    for (uint32_t spin = 0; __hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target;
         spin++) {
      if (spin >= kBarrierSpins) {
        atomicOr(err, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

__global__ __launch_bounds__(256) void k_small_rounds(SmallRounds S, Pyramid P, CamCrit cc, WantParams wp) {
  __shared__ uint32_t ws[kScanThreads / 64];
  __shared__ int s_ok;
  const int64_t nb = gridDim.x, b = blockIdx.x;
  uint32_t nbar = 0, last = 0, rounds = 0, conv = 0;
  int src = 0;
  int64_t cur = S.cur0;
  while (cur <= S.cap / 2) {
    const int64_t chunk = ((cur + nb - 1) / nb + 255) / 256 * 256;
    const int64_t lo = b * chunk, hi = min(cur, lo + chunk);
    const uint64_t* ids = S.ids[src];
    const uint64_t* verts = S.verts[src];
    uint8_t* flags = S.flags[src];
    // mark
    uint32_t part = 0;
    for (int64_t base = lo; base < hi; base += 256) {
      const int64_t i = base + threadIdx.x;
      if (i < hi) {
        uint64_t v[4] = {verts[4 * i], verts[4 * i + 1], verts[4 * i + 2], verts[4 * i + 3]};
        const uint8_t fl = flags[i];
        bool split = false;
        if (!(fl & 1)) {
          if (want(P, cc, wp, v, ids[i])) split = true;
          else flags[i] = 1;
        }
        if (!split) split = hanging(v, S.vset, S.vmask);
        S.cnt[i] = split ? 2u : 1u;
        part += split ? 2u : 1u;
      }
    }
    uint32_t btot;
    block_exclusive(part, ws, &btot);
    if (threadIdx.x == 0) S.bsum[b] = btot;
    if (!grid_barrier(&S.state[4], &S.state[5], ++nbar, &s_ok)) return;
    // output offset of this block and the new leaf count
    uint32_t pre = 0, tot = 0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) {
      const uint32_t x = S.bsum[k];
      tot += x;
      if (k < b) pre += x;
    }
    uint32_t bpre, btot2;
    block_exclusive(pre, ws, &bpre);
    block_exclusive(tot, ws, &btot2);
    pre = bpre;
    tot = btot2;
    if ((int64_t)tot == cur) {
      conv = 1;
      break;
    }
    // split
    uint32_t carry = pre;
    for (int64_t base = lo; base < hi; base += 256) {
      const int64_t i = base + threadIdx.x;
      const uint32_t x = i < hi ? S.cnt[i] : 0u;
      uint32_t t;
      const uint32_t ex = block_exclusive(x, ws, &t);
      bool added = false;
      if (i < hi)
        added = split_one(i, (int64_t)carry + ex, x != 1u, ids, verts, flags, S.chain[src], S.ids[src ^ 1],
                          S.verts[src ^ 1], S.flags[src ^ 1], S.chain[src ^ 1], S.vset, S.vmask, nullptr, 0,
                          nullptr, S.work);
      block_count(added, S.vcount);
      carry += t;
    }
    if (!grid_barrier(&S.state[4], &S.state[5], ++nbar, &s_ok)) return;
    last = (uint32_t)(tot - cur);
    cur = tot;
    src ^= 1;
    rounds++;
  }
  if (b == 0 && threadIdx.x == 0) {
    S.state[0] = (uint32_t)cur;
    S.state[1] = rounds;
    S.state[2] = last;
    S.state[3] = conv;
  }
}

// ---------------------------------------------------------------- finalize
__global__ void k_keys(int64_t n, const uint64_t* __restrict__ ids, uint64_t* __restrict__ keys, int* maxd) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int d = 0;
  if (i < n) {
    uint64_t id = ids[i];
    d = id_depth(id);
    keys[i] = id << (60 - d);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d = max(d, __shfl_xor(d, off, 64));
  // block maximum, then one atomic per block, skipped when it cannot raise
  // the running maximum (one address: contended atomics would serialise)
  __shared__ int s_max[16];
  const int w = threadIdx.x >> 6;
  if (__lane_id() == 0) s_max[w] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = s_max[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) m = max(m, s_max[k]);
    if (m > __hip_atomic_load(maxd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(maxd, m);
  }
}

// kidx[b] = first index whose key is in bucket b or later (a lower-bound
// search per bucket; b = key_buckets gives n).
__global__ void k_key_index(int64_t n, const uint64_t* __restrict__ keys, int kbits, uint32_t* __restrict__ kidx) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = key_buckets(kbits);
  if (b > nb) return;
  if (b == nb) {
    kidx[b] = (uint32_t)n;
    return;
  }
  const uint64_t first = ((8ull << kbits) + (uint64_t)b) << (60 - kbits);
  int64_t lo = 0, hi = n;  // first index with keys >= first
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < first) lo = mid + 1;
    else hi = mid;
  }
  kidx[b] = (uint32_t)lo;
}

// Root Kuhn tets: vertex 1 = S e_p0, vertex 2 = S (e_p0 + e_p1), over the
// axis orders (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1), (2,1,0).
__device__ inline void root_verts(int r, int32_t v[4][3]) {
  const int p0[6] = {0, 0, 1, 1, 2, 2}, p1[6] = {1, 2, 0, 2, 0, 1};
#pragma unroll
  for (int j = 0; j < 4; j++)
#pragma unroll
    for (int a = 0; a < 3; a++) v[j][a] = j == 3 ? kLatS : 0;
  for (int a = 0; a < 3; a++) {
    if (a == p0[r]) { v[1][a] = kLatS; v[2][a] = kLatS; }
    if (a == p1[r]) v[2][a] = kLatS;
  }
}

__device__ inline int isgn(int64_t x) { return (x > 0) - (x < 0); }

// Bisection step of the perturbed-point descent for a compile-time tag K:
// the point is 3 * face centroid (q3, below 2^22) plus epsilon * outward
// normal.
template <int K>
__device__ inline void descend_perturbed(int32_t v[4][3], uint64_t& h, uint32_t& cls, const uint32_t* __restrict__ shapes,
                                         const int32_t q3[3], const int nout[3]) {
  const uint32_t w = shapes[cls];
  int32_t z[3], u[3];
  shape_bisector<K>(v, w, z, u);
  int32_t side = 0, pert = 0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    side += __mul24(u[i], q3[i] - 3 * z[i]);
    pert += __mul24(u[i], nout[i]);
  }
  bool first = side != 0 ? side > 0 : pert > 0;
  cls = first ? (w >> 8) & 255u : (w >> 16) & 255u;
  if (first) {
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

// Outward unit normal of the face (a, b, c) opposite vertex o and its
// lattice offset; returns false when the normal is not one of the 18
// orientations.
__device__ inline bool face_normal(const int64_t a[3], const int64_t b[3], const int64_t c[3], const int64_t o[3],
                                   int un[3], int64_t& off) {
  int64_t e1[3], e2[3], n[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    e1[i] = b[i] - a[i];
    e2[i] = c[i] - a[i];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < 3; i++) s += n[i] * (o[i] - a[i]);
  if (s == 0) return false;
  int64_t m = 0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    if (s > 0) n[i] = -n[i];
    int64_t ab = n[i] < 0 ? -n[i] : n[i];
    m = ab > m ? ab : m;
  }
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    int64_t ab = n[i] < 0 ? -n[i] : n[i];
    if (ab != 0 && ab != m) ok = false;
    un[i] = isgn(n[i]);
  }
  int nz = (un[0] != 0) + (un[1] != 0) + (un[2] != 0);
  if (nz > 2) ok = false;
  off = un[0] * a[0] + un[1] * a[1] + un[2] * a[2];
  return ok;
}

// Element i of a 4-array held in registers (selects, no indexed access).
template <class T>
__device__ inline T pick4(const T x[4], int i) {
  return i == 0 ? x[0] : (i == 1 ? x[1] : (i == 2 ? x[2] : x[3]));
}

// Kuhn root whose axis order sorts the point (q3, perturbed along un) in
// descending order: pairwise comparisons of (q3, un), lexicographic; -1 on
// a tie.
__device__ inline int root_of(const int64_t q3[3], const int un[3]) {
  auto cmp = [&](int a, int b) {
    const int c = isgn(q3[a] - q3[b]);
    return c ? c : isgn((int64_t)un[a] - un[b]);
  };
  const int c01 = cmp(0, 1), c02 = cmp(0, 2), c12 = cmp(1, 2);
  if (!c01 || !c02 || !c12) return -1;
  // axis orders (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1), (2,1,0)
  if (c01 > 0 && c12 > 0) return 0;
  if (c02 > 0 && c12 < 0) return c01 > 0 ? 1 : -1;
  if (c01 < 0 && c02 > 0) return 2;
  if (c12 > 0 && c02 < 0) return c01 < 0 ? 3 : -1;
  if (c02 < 0 && c01 > 0) return 4;
  return 5;
}

// Face f of the tet v: its three vertices (the others, in order) and the
// opposite vertex (selects keep the arrays in registers).
__device__ inline void face_of(const int64_t v[4][3], int f, int64_t fa[3], int64_t fb[3], int64_t fc[3],
                               int64_t fo[3]) {
  const int i0 = f == 0 ? 1 : 0, i1 = f <= 1 ? 2 : 1, i2 = f <= 2 ? 3 : 2;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const int64_t col[4] = {v[0][a], v[1][a], v[2][a], v[3][a]};
    fa[a] = pick4(col, i0);
    fb[a] = pick4(col, i1);
    fc[a] = pick4(col, i2);
    fo[a] = pick4(col, f);
  }
}

__device__ inline void unpack_tet(const uint64_t* __restrict__ verts, int64_t t, uint64_t pv[4], int64_t v[4][3]) {
#pragma unroll
  for (int j = 0; j < 4; j++) {
    pv[j] = verts[4 * t + j];
    v[j][0] = vx(pv[j]);
    v[j][1] = vy(pv[j]);
    v[j][2] = vz(pv[j]);
  }
}

// Records, first pass (one thread per tet): extinction, majorant, face
// planes and codes, boundary links.  Interior faces are linked from one
// side only: the two tets on a face see it with opposite outward normals,
// and the tet that sees +dir_N (orientation bit 0) lists the face as
// (t << 2 | f) for k_links, so every face is searched once and the
// searches run on full waves.  One atomic per block for the list positions.
constexpr int kRecordsBlock = 1024;

__global__ __launch_bounds__(kRecordsBlock) void k_records(int64_t n, const uint64_t* __restrict__ verts, Pyramid P,
                                                           float scale, int majorant_mode, TetRec* __restrict__ rec,
                                                           TetRec32* __restrict__ rec32, uint32_t* __restrict__ items,
                                                           int64_t item_cap, uint32_t* item_count,
                                                           int* __restrict__ err) {
  __shared__ uint32_t s_wave[kRecordsBlock / 64], s_base;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t owned = 0;  // bit f: this tet links face f
  if (t < n) {
    uint64_t pv[4];
    int64_t v[4][3];
    unpack_tet(verts, t, pv, v);
    // medium: extinction = scale * mean(D), majorant tight or scale * max(D)
    int32_t lo[3], hi[3];
    tet_box(pv, lo, hi);
    float mn, mx;
    double s, c;
    box_stats(P, lo, hi, mn, mx, s, c);
    const double mean = s / c;
    const float sigma = (float)((double)scale * mean);
    const float majorant = majorant_mode == 1 ? (float)((double)scale * (double)mx) : sigma;
    uint32_t codes = 0;
    float offs[4];
    int32_t ioff[4];
#pragma unroll 1
    for (int f = 0; f < 4; f++) {
      int64_t fa3[3], fb3[3], fc3[3], fo3[3];
      face_of(v, f, fa3, fb3, fc3, fo3);
      int un[3];
      int64_t off;
      int code = -1;
      if (face_normal(fa3, fb3, fc3, fo3, un, off)) code = dir_code(un);
      if (code < 0) {
        atomicOr(err, 2);
        code = 0;
      }
      codes |= (uint32_t)code << (8 * f);
      // boundary face: its three vertices share a coordinate equal to 0 or S
      bool bnd = false;
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const int64_t x = fa3[a];
        if (fb3[a] == x && fc3[a] == x && (x == 0 || x == kLatS)) bnd = true;
      }
      if (bnd) {
        rec[t].nbr[f] = kBoundary;
        if (rec32) rec32[t].w[4 + f] = kLink27Boundary | code_bits32((uint32_t)code);
      } else if (!(code & 1)) {
        owned |= 1u << f;
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (k == f) {
          offs[k] = ldexpf((float)off, -kLatBits);
          ioff[k] = (int32_t)off;
        }
      }
    }
    // the record's other words (link words: above, or by k_links)
    reinterpret_cast<float4*>(&rec[t])[0] = make_float4(offs[0], offs[1], offs[2], offs[3]);
    reinterpret_cast<uint4*>(&rec[t])[2] =
        make_uint4(codes, __float_as_uint(sigma), __float_as_uint(majorant), 0u);
    if (rec32) {
      uint64_t lo64 = ((uint64_t)(ioff[0] & 0x7FFFFF)) | ((uint64_t)(ioff[1] & 0x7FFFFF) << 23) |
                      ((uint64_t)(ioff[2] & 0x3FFFF) << 46);
      uint64_t hi64 = ((uint64_t)(ioff[2] & 0x7FFFFF) >> 18) | ((uint64_t)(ioff[3] & 0x7FFFFF) << 5);
      reinterpret_cast<uint4*>(&rec32[t])[0] =
          make_uint4((uint32_t)lo64, (uint32_t)(lo64 >> 32), (uint32_t)hi64, __float_as_uint(sigma));
    }
  }
  // list positions: block prefix of the counts, one atomic per block
  const uint32_t x = __popc(owned);
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_wave[wid] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < kRecordsBlock / 64; w++) {
      const uint32_t c = s_wave[w];
      s_wave[w] = run;
      run += c;
    }
    s_base = run ? atomicAdd(item_count, run) : 0u;
  }
  __syncthreads();
  int64_t pos = (int64_t)s_base + s_wave[wid] + (inc - x);
#pragma unroll 1
  for (int f = 0; f < 4; f++) {
    if (!((owned >> f) & 1u)) continue;
    if (pos < item_cap) items[pos] = ((uint32_t)t << 2) | (uint32_t)f;
    else atomicOr(err, 8);  // more interior faces than a conforming grid has
    pos++;
  }
}

// Records, second pass (one thread per listed face): the neighbour across
// face f of tet t, from the tet holding a point just outside the face (the
// face centroid pushed outward by a symbolic epsilon: exact descent, then
// the key search), checked to share the face; writes both link words.
__global__ void k_links(const uint32_t* __restrict__ items, const uint32_t* __restrict__ item_count, int64_t item_cap,
                        int64_t n,
                        const uint64_t* __restrict__ verts, const uint64_t* __restrict__ keys,
                        const uint32_t* __restrict__ kidx, int kbits, int dmax, const uint32_t* __restrict__ shapes,
                        TetRec* __restrict__ rec, TetRec32* __restrict__ rec32, int* __restrict__ err) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= min((int64_t)*item_count, item_cap)) return;
  const uint32_t it = items[s];
  const int64_t t = it >> 2;
  const int f = (int)(it & 3u);
  uint64_t pv[4];
  int64_t v[4][3];
  unpack_tet(verts, t, pv, v);
  int64_t fa3[3], fb3[3], fc3[3], fo3[3];
  face_of(v, f, fa3, fb3, fc3, fo3);
  int un[3];
  int64_t off;
  int code = 0;
  if (face_normal(fa3, fb3, fc3, fo3, un, off)) code = max(dir_code(un), 0);
  uint32_t link = kBoundary;
  int64_t q3[3];
#pragma unroll
  for (int a = 0; a < 3; a++) q3[a] = fa3[a] + fb3[a] + fc3[a];
  const int root = root_of(q3, un);
  if (root < 0) {
    atomicOr(err, 4);
  } else {
    int32_t w[4][3], q3i[3] = {(int32_t)q3[0], (int32_t)q3[1], (int32_t)q3[2]};
    root_verts(root, w);
    uint64_t h = 8 + root;
    uint32_t cls = shapes[kShapeWords + root];
    for (int d = 0; d < dmax; d += 3) {
      descend_perturbed<3>(w, h, cls, shapes, q3i, un);
      if (d + 1 < dmax) descend_perturbed<2>(w, h, cls, shapes, q3i, un);
      if (d + 2 < dmax) descend_perturbed<1>(w, h, cls, shapes, q3i, un);
    }
    const int64_t nb = search_keys_idx(keys, kidx, kbits, h << (60 - dmax));
    // back face: the neighbour's vertex that is not on face f
    const int i0 = f == 0 ? 1 : 0, i1 = f <= 1 ? 2 : 1, i2 = f <= 2 ? 3 : 2;
    const uint64_t fa = pick4(pv, i0), fb = pick4(pv, i1), fc = pick4(pv, i2);
    int bf = -1, hits = 0;
    if (nb >= 0 && nb < n) {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const uint64_t x = verts[4 * nb + j];
        if (x == fa || x == fb || x == fc) hits++;
        else bf = j;
      }
    }
    if (nb < 0 || nb >= n || nb == t || hits != 3 || bf < 0) {
      atomicOr(err, 1);
    } else {
      link = ((uint32_t)nb << 2) | (uint32_t)bf;
      // the neighbour sees this face as -dir_N across its face bf
      rec[nb].nbr[bf] = ((uint32_t)t << 2) | (uint32_t)f;
      if (rec32) rec32[nb].w[4 + bf] = (uint32_t)t | code_bits32((uint32_t)(code ^ 1));
    }
  }
  rec[t].nbr[f] = link;
  if (rec32) rec32[t].w[4 + f] = (link == kBoundary ? kLink27Boundary : (link >> 2)) | code_bits32((uint32_t)code);
}

// ---------------------------------------------------------------- host
static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- shape classes
// The classes are found by bisecting, from the six roots, one
// representative of each class (x_0 = 0, x_j = 4 e_j with e_j the class's
// reduced edge vectors, so midpoints stay integral) until no new class
// appears; normals come from exact integer cross products.
namespace {
struct ShapeKey {
  std::array<int64_t, 9> e;
  int tag;
  bool operator<(const ShapeKey& o) const { return tag != o.tag ? tag < o.tag : e < o.e; }
};

ShapeKey shape_key(const int64_t v[4][3], int tag) {
  ShapeKey k;
  int64_t m = 0;
  for (int j = 1; j < 4; j++)
    for (int i = 0; i < 3; i++) {
      k.e[3 * (j - 1) + i] = v[j][i] - v[0][i];
      m |= k.e[3 * (j - 1) + i];
    }
  const int sh = m ? __builtin_ctzll((uint64_t)m) : 0;
  for (auto& x : k.e) x >>= sh;
  k.tag = tag;
  return k;
}

bool make_shapes(std::vector<uint32_t>& tab) {
  tab.assign(kShapeWords + 8, 0u);
  std::map<ShapeKey, int> ids;
  std::vector<ShapeKey> reps;
  auto intern = [&](const int64_t v[4][3], int tag) {
    ShapeKey k = shape_key(v, tag);
    auto it = ids.find(k);
    if (it != ids.end()) return it->second;
    const int c = (int)reps.size();
    ids.emplace(k, c);
    reps.push_back(k);
    return c;
  };
  const int p0[6] = {0, 0, 1, 1, 2, 2}, p1[6] = {1, 2, 0, 2, 0, 1};
  for (int r = 0; r < 6; r++) {
    int64_t v[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {kLatS, kLatS, kLatS}};
    v[1][p0[r]] = kLatS;
    v[2][p0[r]] = kLatS;
    v[2][p1[r]] = kLatS;
    tab[kShapeWords + r] = (uint32_t)intern(v, 3);
  }
  for (size_t c = 0; c < reps.size(); c++) {
    if (reps.size() > (size_t)kShapeWords) return false;
    const ShapeKey k = reps[c];
    const int K = k.tag, J1 = K == 1 ? 2 : 1, J2 = K == 3 ? 2 : 3;
    int64_t v[4][3] = {{0, 0, 0}};
    for (int j = 1; j < 4; j++)
      for (int i = 0; i < 3; i++) v[j][i] = 4 * k.e[3 * (j - 1) + i];
    int64_t z[3], a[3], b[3], d[3], n[3];
    for (int i = 0; i < 3; i++) {
      z[i] = (v[0][i] + v[K][i]) / 2;
      a[i] = v[J1][i] - z[i];
      b[i] = v[J2][i] - z[i];
      d[i] = v[0][i] - z[i];
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    const int64_t s0 = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    if (s0 == 0) return false;
    uint32_t w = 0;
    for (int i = 0; i < 3; i++) {
      int u = (n[i] > 0) - (n[i] < 0);
      if (s0 < 0) u = -u;
      w |= (uint32_t)(u + 1) << (2 * i);
    }
    // first child: x_K -> z; second child: (x_1..x_K, z, x_{K+1}..x_3)
    const int ctag = K == 1 ? 3 : K - 1;
    int64_t ca[4][3], cb[4][3];
    for (int j = 0; j < 4; j++)
      for (int i = 0; i < 3; i++) ca[j][i] = j == K ? z[i] : v[j][i];
    for (int j = 0; j < 4; j++)
      for (int i = 0; i < 3; i++) cb[j][i] = j < K ? v[j + 1][i] : (j == K ? z[i] : v[j][i]);
    const int ia = intern(ca, ctag), ib = intern(cb, ctag);
    w |= (uint32_t)ia << 8 | (uint32_t)ib << 16;
    tab[c] = w;
  }
  return reps.size() <= (size_t)kShapeWords;
}
}  // namespace

namespace {
std::mutex g_shape_mu;
std::map<int, uint32_t*> g_shape_tab;  // one copy per device, kept until exit
}  // namespace

const uint32_t* shape_table_existing() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  auto it = g_shape_tab.find(dev);
  return it == g_shape_tab.end() ? nullptr : it->second;
}

const uint32_t* shape_table() {
  static std::once_flag once;
  static std::vector<uint32_t> host;
  static bool ok = false;
  std::call_once(once, [] { ok = make_shapes(host); });
  if (!ok) return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  auto& dev_tab = g_shape_tab;
  auto it = dev_tab.find(dev);
  if (it != dev_tab.end()) return it->second;
  uint32_t* p = nullptr;
  if (hipMalloc((void**)&p, host.size() * 4) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipMemcpy(p, host.data(), host.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p);
    return nullptr;
  }
  dev_tab.emplace(dev, p);
  return p;
}

namespace {
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { release(); }
  void swap_with(Buf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  bool ensure(size_t b) {
    if (b <= bytes) return true;
    release();
    size_t nb = std::max<size_t>(b, 256);
    p = dev_alloc(nb);
    if (!p) return false;
    bytes = nb;
    return true;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

struct Leaves {
  Buf ids, verts, flags, chain;
  int64_t cap = 0;
  void swap_with(Leaves& o) {
    ids.swap_with(o.ids);
    verts.swap_with(o.verts);
    flags.swap_with(o.flags);
    chain.swap_with(o.chain);
    std::swap(cap, o.cap);
  }
  bool ensure(int64_t n) {
    if (n <= cap) return true;
    int64_t c = std::max<int64_t>(n, cap + cap / 2);
    if (!ids.ensure(c * 8) || !verts.ensure(c * 32) || !flags.ensure(c) || !chain.ensure(c * 8)) return false;
    cap = c;
    return true;
  }
  // Room for n leaves, keeping the first `keep` (copied on the stream, which
  // is drained before the old arrays return to the pool).
  bool grow_keep(int64_t n, int64_t keep, hipStream_t st) {
    if (n <= cap) return true;
    Leaves t;
    if (!t.ensure(std::max<int64_t>(n, cap + cap / 4))) return false;
    if (keep > 0 && (hipMemcpyAsync(t.ids.p, ids.p, keep * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                     hipMemcpyAsync(t.verts.p, verts.p, keep * 32, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                     hipMemcpyAsync(t.flags.p, flags.p, keep, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                     hipMemcpyAsync(t.chain.p, chain.p, keep * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                     hipStreamSynchronize(st) != hipSuccess))
      return false;
    swap_with(t);
    return true;
  }
};

// Min / max / FP64-sum pyramid of an n^3 grid (n = 2^L) on the device,
// levels 1..L in lv; false when out of memory.
static bool make_pyramid(const float* d, int32_t n, int L, Pyramid& P, std::vector<Buf>& lv, hipStream_t st) {
  memset(&P, 0, sizeof(P));
  P.dens = d;
  P.n = n;
  P.L = L;
  lv = std::vector<Buf>(3 * (L + 1));
  for (int l = 1; l <= L; l++) {
    int64_t m = (int64_t)n >> l, cells = m * m * m;
    if (!lv[3 * l].ensure(cells * 4) || !lv[3 * l + 1].ensure(cells * 4) || !lv[3 * l + 2].ensure(cells * 8))
      return false;
    P.mn[l] = lv[3 * l].as<float>();
    P.mx[l] = lv[3 * l + 1].as<float>();
    P.sum[l] = lv[3 * l + 2].as<double>();
    hipLaunchKernelGGL(k_pyramid_level, dim3(nblocks(cells, 256)), dim3(256), 0, st, l == 1 ? d : nullptr,
                       l == 1 ? nullptr : P.mn[l - 1], l == 1 ? nullptr : P.mx[l - 1],
                       l == 1 ? nullptr : P.sum[l - 1], (int32_t)m, (float*)P.mn[l], (float*)P.mx[l],
                       (double*)P.sum[l]);
  }
  return true;
}

// Sparse volume: brick map (bit 1 of *bad: a coordinate out of range, bit 2:
// a brick listed twice).
__global__ void k_brick_map(const int32_t* __restrict__ coords, int64_t nbricks, int32_t nb, int32_t* __restrict__ bmap,
                            int* __restrict__ bad) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbricks) return;
  const int32_t x = coords[3 * b], y = coords[3 * b + 1], z = coords[3 * b + 2];
  if (x < 0 || y < 0 || z < 0 || x >= nb || y >= nb || z >= nb) {
    atomicOr(bad, 2);
    return;
  }
  if (atomicCAS(&bmap[x + (int64_t)nb * (y + (int64_t)nb * z)], -1, (int32_t)b) != -1) atomicOr(bad, 4);
}

// One wave per brick: levels 1 (64 cells) and 2 (8 cells) of the brick, and
// its level-3 cell in the dense level-3 arrays; children combined as in
// k_pyramid_level.
__global__ __launch_bounds__(64) void k_brick_levels(const int32_t* __restrict__ coords, const float* __restrict__ val,
                                                     int32_t nb, float* __restrict__ mn1, float* __restrict__ mx1,
                                                     double* __restrict__ s1, float* __restrict__ mn2,
                                                     float* __restrict__ mx2, double* __restrict__ s2,
                                                     float* __restrict__ mn3, float* __restrict__ mx3,
                                                     double* __restrict__ s3) {
  __shared__ float lmn[64], lmx[64];
  __shared__ double lsum[64];
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x;
  auto combine = [](const float* lo, const float* hi, const double* s, float& a, float& c, double& sum) {
    a = lo[0];
    c = hi[0];
    for (int q = 1; q < 8; q++) {
      a = lo[q] < a ? lo[q] : a;
      c = hi[q] > c ? hi[q] : c;
    }
    sum = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  };
  {  // level 1: cell (i, j, k) of 4^3 from voxels (2i + a, 2j + b, 2k + c) of 8^3
    const int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
    float lo[8], hi[8];
    double s[8];
    for (int q = 0; q < 8; q++) {
      const float v = val[b * 512 + (2 * i + (q & 1)) + 8 * ((2 * j + ((q >> 1) & 1)) + 8 * (2 * k + ((q >> 2) & 1)))];
      lo[q] = v;
      hi[q] = v;
      s[q] = (double)v;
    }
    float a, c;
    double sum;
    combine(lo, hi, s, a, c, sum);
    mn1[b * 64 + t] = a;
    mx1[b * 64 + t] = c;
    s1[b * 64 + t] = sum;
    lmn[t] = a;
    lmx[t] = c;
    lsum[t] = sum;
  }
  __syncthreads();
  float a2 = 0.0f, c2 = 0.0f;
  double sum2 = 0.0;
  if (t < 8) {  // level 2: cell of 2^3 from level-1 cells of 4^3
    const int i = t & 1, j = (t >> 1) & 1, k = t >> 2;
    float lo[8], hi[8];
    double s[8];
    for (int q = 0; q < 8; q++) {
      const int c = (2 * i + (q & 1)) + 4 * ((2 * j + ((q >> 1) & 1)) + 4 * (2 * k + ((q >> 2) & 1)));
      lo[q] = lmn[c];
      hi[q] = lmx[c];
      s[q] = lsum[c];
    }
    combine(lo, hi, s, a2, c2, sum2);
    mn2[b * 8 + t] = a2;
    mx2[b * 8 + t] = c2;
    s2[b * 8 + t] = sum2;
  }
  __syncthreads();
  if (t < 8) {
    lmn[t] = a2;
    lmx[t] = c2;
    lsum[t] = sum2;
  }
  __syncthreads();
  const int32_t bx = coords[3 * b], by = coords[3 * b + 1], bz = coords[3 * b + 2];
  if (t == 0 && bx >= 0 && by >= 0 && bz >= 0 && bx < nb && by < nb && bz < nb) {
    // level 3: the brick's own cell (child order q = x + 2y + 4z); bricks
    // out of range are reported by k_brick_map and skipped here
    float a, c;
    double sum;
    combine(lmn, lmx, lsum, a, c, sum);
    const int64_t o = bx + (int64_t)nb * (by + (int64_t)nb * bz);
    mn3[o] = a;
    mx3[o] = c;
    s3[o] = sum;
  }
}

// Pyramid of a sparse volume (n >= 8): brick map, per-brick levels 1-2,
// dense levels 3..L (level 3 zero where no brick).  Bricks and values on
// the device; *d_bad gets bits 2 / 4 for bad coordinates / duplicates.
static bool make_sparse_pyramid(const int32_t* coords, const float* val, int64_t nbricks, int32_t n, int L, Pyramid& P,
                                std::vector<Buf>& lv, int* d_bad, hipStream_t st) {
  memset(&P, 0, sizeof(P));
  P.n = n;
  P.L = L;
  const int32_t nb = n >> kBrickBits;
  P.nb = nb;
  const int64_t nbc = (int64_t)nb * nb * nb;
  lv = std::vector<Buf>(3 * (L + 1) + 1);
  Buf& map = lv[3 * (L + 1)];
  if (!map.ensure(nbc * 4)) return false;
  hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(nbc, 256)), dim3(256), 0, st, map.as<uint32_t>(), nbc, 0xFFFFFFFFu);
  if (nbricks > 0)
    hipLaunchKernelGGL(k_brick_map, dim3(nblocks(nbricks, 256)), dim3(256), 0, st, coords, nbricks, nb,
                       map.as<int32_t>(), d_bad);
  P.bmap = map.as<int32_t>();
  P.bval = val;
  const int64_t nbr = std::max<int64_t>(nbricks, 1);
  for (int l = 1; l <= 2; l++) {  // per-brick levels
    const int64_t cells = nbr * (l == 1 ? 64 : 8);
    if (!lv[3 * l].ensure(cells * 4) || !lv[3 * l + 1].ensure(cells * 4) || !lv[3 * l + 2].ensure(cells * 8))
      return false;
    P.bmn[l] = lv[3 * l].as<float>();
    P.bmx[l] = lv[3 * l + 1].as<float>();
    P.bsum[l] = lv[3 * l + 2].as<double>();
  }
  for (int l = 3; l <= L; l++) {
    const int64_t m = (int64_t)n >> l, cells = m * m * m;
    if (!lv[3 * l].ensure(cells * 4) || !lv[3 * l + 1].ensure(cells * 4) || !lv[3 * l + 2].ensure(cells * 8))
      return false;
    P.mn[l] = lv[3 * l].as<float>();
    P.mx[l] = lv[3 * l + 1].as<float>();
    P.sum[l] = lv[3 * l + 2].as<double>();
    if (l == 3) {
      if (hipMemsetAsync(lv[9].p, 0, cells * 4, st) != hipSuccess ||
          hipMemsetAsync(lv[10].p, 0, cells * 4, st) != hipSuccess ||
          hipMemsetAsync(lv[11].p, 0, cells * 8, st) != hipSuccess)
        return false;
      if (nbricks > 0)
        hipLaunchKernelGGL(k_brick_levels, dim3((unsigned)nbricks), dim3(64), 0, st, coords, val, nb,
                           (float*)P.bmn[1], (float*)P.bmx[1], (double*)P.bsum[1], (float*)P.bmn[2], (float*)P.bmx[2],
                           (double*)P.bsum[2], (float*)P.mn[3], (float*)P.mx[3], (double*)P.sum[3]);
    } else {
      hipLaunchKernelGGL(k_pyramid_level, dim3(nblocks(cells, 256)), dim3(256), 0, st, nullptr, P.mn[l - 1],
                         P.mx[l - 1], P.sum[l - 1], (int32_t)m, (float*)P.mn[l], (float*)P.mx[l], (double*)P.sum[l]);
    }
  }
  return true;
}

// A device buffer grown keeping its first `keep` bytes.
static bool grow_keep(Buf& b, size_t bytes, size_t keep, hipStream_t st) {
  if (bytes <= b.bytes) return true;
  Buf t;
  if (!t.ensure(std::max(bytes, b.bytes + b.bytes / 4))) return false;
  if (keep > 0 && (hipMemcpyAsync(t.p, b.p, keep, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess))
    return false;
  b.swap_with(t);
  return true;
}
}  // namespace

static int64_t scan_u32(const uint32_t* in, int64_t n, uint32_t* out, Buf& bsum, uint32_t* d_total, hipStream_t st) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (!bsum.ensure(nb * 4)) return -1;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, bsum.as<uint32_t>());
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, bsum.as<uint32_t>(), nb, d_total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, bsum.as<uint32_t>(), out);
  return 0;
}

// The build from a dense volume (dens) or a sparse one (sp): they differ
// only in how the pyramid is made.
// The seed of a build from a previous grid (see k_seed_chain): its leaves in
// A (depth-first order), the wanted ones listed in wk, its vertices in a new
// vertex set vs of *vcap keys.  *cur and *nwork receive the counts;
// *unchanged is set (and nothing else done) when the previous grid is
// already the result.
static int seed_from_grid(const tet_grid* prev, const Pyramid& P, const CamCrit& cc, const WantParams& wp,
                          Leaves& A, Buf& wk, Buf& vs, uint64_t* vcap, Buf& bsum, uint32_t* d_total,
                          uint32_t* d_count, uint32_t* d_vcount, uint32_t* hbuf, hipStream_t st, int64_t* cur,
                          int64_t* nwork, bool allow_same, bool* unchanged) {
  const int64_t n = prev->n;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  *unchanged = false;
  Buf keep, bits, first, pos, bagg;
  if (!keep.ensure(n * 8) || !bits.ensure(n * 8) || !first.ensure(n * 4) || !pos.ensure(n * 4) ||
      !bagg.ensure(nb * sizeof(ChainT)))
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_update: seed");
  hipLaunchKernelGGL(k_seed_chain, dim3(nblocks(n, 256)), dim3(256), 0, st, n, (const uint64_t*)prev->ids, P, cc, wp,
                     keep.as<uint64_t>(), bits.as<uint64_t>());
  hipLaunchKernelGGL(k_chain_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, keep.as<uint64_t>(),
                     bits.as<uint64_t>(), n, bagg.as<ChainT>());
  hipLaunchKernelGGL(k_chain_blocks, dim3(1), dim3(kScanThreads), 0, st, bagg.as<ChainT>(), nb);
  hipLaunchKernelGGL(k_chain_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, keep.as<uint64_t>(),
                     bits.as<uint64_t>(), n, bagg.as<ChainT>());
  if (allow_same) {
    TV_HIP(hipMemsetAsync(d_count, 0, 4, st));
    hipLaunchKernelGGL(k_chain_diff, dim3(nblocks(n, 256)), dim3(256), 0, st, n,
                       (const uint64_t*)bits.as<uint64_t>(), (const uint64_t*)prev->chain, d_count);
    TV_HIP(hipMemcpyAsync(hbuf, d_count, 4, hipMemcpyDeviceToHost, st));
    TV_HIP(hipStreamSynchronize(st));
    if (hbuf[0] == 0) {
      *unchanged = true;
      return TET_OK;
    }
  }
  hipLaunchKernelGGL(k_seed_first, dim3(nblocks(n, 256)), dim3(256), 0, st, n, (const uint64_t*)prev->ids,
                     bits.as<uint64_t>(), first.as<uint32_t>());
  if (scan_u32(first.as<uint32_t>(), n, pos.as<uint32_t>(), bsum, d_total, st))
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_update: seed scan");
  TV_HIP(hipMemcpyAsync(hbuf, d_total, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  const int64_t m = hbuf[0];
  if (m < 6 || m > n) return fail(TET_ERR_INTERNAL, "leb_update: bad seed size");
  if (!A.ensure(std::max<int64_t>(m, 1 << 16)) || !wk.ensure((size_t)m * 4))
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_update: seed leaves");
  // a seed holds the 8 corners and at most one vertex per split node (m - 6
  // of them); the set stays at most half full
  uint64_t cap = 1 << 16;
  while (cap < 2 * (uint64_t)(m + 2)) cap <<= 2;
  if (!vs.ensure(cap * 8)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_update: vertex set");
  hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(cap, 256)), dim3(256), 0, st, vs.as<uint64_t>(), (int64_t)cap,
                     kEmptyKey);
  TV_HIP(hipMemsetAsync(d_count, 0, 4, st));
  hipLaunchKernelGGL(k_seed_write, dim3(nblocks(n, 256)), dim3(256), 0, st, n, (const uint64_t*)prev->ids,
                     bits.as<uint64_t>(), first.as<uint32_t>(), pos.as<uint32_t>(), A.ids.as<uint64_t>(),
                     A.verts.as<uint64_t>(), A.flags.as<uint8_t>(), A.chain.as<uint64_t>(), wk.as<uint32_t>(), d_count,
                     vs.as<uint64_t>(), cap - 1, d_vcount);
  TV_HIP(hipGetLastError());
  TV_HIP(hipMemcpyAsync(hbuf, d_count, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));  // before the scratch returns to the pool
  *cur = m;
  *nwork = hbuf[0];
  *vcap = cap;
  return TET_OK;
}

static int build_common(const tet_density* dens, const tet_sparse_density* sp, const tet_camera* cam, float target_px,
                        const tet_build_opts* opts_in, hipStream_t st, tet_grid** out,
                        tet_grid* prev = nullptr, float* unchanged_ms = nullptr) {
  if (!out) return fail(TET_ERR_INVALID_ARG, "leb_build: out is NULL");
  *out = nullptr;
  const int32_t n = sp ? sp->n : dens->n;
  const float scale = sp ? sp->density_scale : dens->density_scale;
  if (n < 1 || n > 4096 || (n & (n - 1))) return fail(TET_ERR_INVALID_ARG, "leb_build: n must be a power of two <= 4096");
  if (sp && n < (1 << kBrickBits)) return fail(TET_ERR_INVALID_ARG, "leb_build_sparse: n must be at least 8");
  if (int rc = check_camera(cam)) return rc;
  tet_build_opts o;
  if (opts_in) o = *opts_in;
  else tet_build_opts_defaults(&o);
  if (o.want_mode < 0 || o.want_mode > 2 || o.max_tets < 6 || o.max_tets > (1ll << 30) || o.max_depth < 0 ||
      o.max_depth > 56 || o.uniform_depth < 0 || o.uniform_depth > 56 || o.majorant_mode < 0 || o.majorant_mode > 1 ||
      o.host_rounds < 0 || o.host_rounds > 1)
    return fail(TET_ERR_INVALID_ARG, "leb_build: bad options");
  if (o.want_mode == 0 && !(target_px > 0.0f)) return fail(TET_ERR_INVALID_ARG, "leb_build: target_cell_px must be > 0");
  if (!(scale >= 0.0f) || std::isinf(scale)) return fail(TET_ERR_INVALID_ARG, "leb_build: bad density_scale");
  if (sp && (sp->num_bricks < 0 || sp->num_bricks > ((int64_t)n * n * n >> (3 * kBrickBits)) ||
             (sp->num_bricks > 0 && (!sp->brick_coords || !sp->brick_values))))
    return fail(TET_ERR_INVALID_ARG, "leb_build_sparse: bad brick list");
  int L = 0;
  while ((1 << L) < n) L++;
  int64_t nvox = (int64_t)n * n * n;

  hipEvent_t e0, e1;
  TV_HIP(hipEventCreate(&e0));
  TV_HIP(hipEventCreate(&e1));
  TV_HIP(hipEventRecord(e0, st));

  // density on the device (a sparse volume: its bricks)
  Buf dcopy, ccopy;
  const float* d_dens = sp ? sp->brick_values : dens->data;
  const int32_t* d_coords = sp ? sp->brick_coords : nullptr;
  const int64_t nbricks = sp ? sp->num_bricks : 0;
  const int64_t nvals = sp ? nbricks << (3 * kBrickBits) : nvox;
  if (!(sp ? sp->on_device : dens->on_device) && nvals > 0) {
    if (!dcopy.ensure(nvals * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: density copy");
    TV_HIP(hipMemcpyAsync(dcopy.p, d_dens, nvals * 4, hipMemcpyHostToDevice, st));
    d_dens = dcopy.as<float>();
    if (sp) {
      if (!ccopy.ensure(nbricks * 12)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: brick copy");
      TV_HIP(hipMemcpyAsync(ccopy.p, d_coords, nbricks * 12, hipMemcpyHostToDevice, st));
      d_coords = ccopy.as<int32_t>();
    }
  }
  // small device scratch (32-bit words): [0] density flag, [1] max depth,
  // [2] finalize error, [3] listed faces, [4] scan total, [5] running count of marked splits,
  // [6, 6 + kCountSlots) vertex count slots, [24, 30) small-round state
  Buf misc;
  if (!misc.ensure(128)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: scratch");
  TV_HIP(hipMemsetAsync(misc.p, 0, 128, st));
  int* d_flag = misc.as<int>();
  uint32_t* d_total = misc.as<uint32_t>() + 4;
  uint32_t* d_splitc = misc.as<uint32_t>() + 5;
  uint32_t* d_vcount = misc.as<uint32_t>() + 6;
  if (nvals > 0)
    hipLaunchKernelGGL(k_check_density, dim3(nblocks(nvals, 256)), dim3(256), 0, st, d_dens, nvals, d_flag);

  // pyramid
  Pyramid P;
  std::vector<Buf> lv;
  if (sp ? !make_sparse_pyramid(d_coords, d_dens, nbricks, n, L, P, lv, d_flag, st)
         : !make_pyramid(d_dens, n, L, P, lv, st))
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: pyramid");
  int flag = 0;
  TV_HIP(hipMemcpyAsync(&flag, d_flag, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  if (flag & 6) return fail(TET_ERR_INVALID_ARG, "leb_build_sparse: brick coordinates out of range or listed twice");
  if (flag) return fail(TET_ERR_NUMERIC, "leb_build: density has NaN, infinite or negative values");

  CamCrit cc;
  make_camcrit(*cam, target_px, &cc);
  WantParams wp;
  memset(&wp, 0, sizeof(wp));
  wp.mode = o.want_mode;
  wp.uniform_depth = o.uniform_depth;
  wp.max_depth = o.max_depth;
  wp.tau = o.variation_tau;
  wp.rand_seed = o.rand_seed;
  wp.rand_thresh = o.rand_thresh;

  // the cooperative launch of the first rounds, where the device supports it
  int coop = 0, ncu = 0, occ = 0, dev = 0;
  TV_HIP(hipGetDevice(&dev));
  TV_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  TV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  TV_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_small_rounds), 256, 0));
  const int64_t small_cap = std::min<int64_t>(kSmallCap, o.max_tets);
  const bool small = !prev && !o.host_rounds && coop && occ > 0 && ncu > 0 && small_cap >= 12;
  // half the CUs: the rounds are small, and every block adds an arrival to
  // each grid barrier (128 blocks measured best on 256 CUs)
  const int small_blocks = std::max(1, ncu / 2);

  uint32_t* hbuf = nullptr;
  TV_HIP(hipHostMalloc((void**)&hbuf, 128, hipHostMallocDefault));
  struct HostFree {
    uint32_t* p;
    ~HostFree() { if (p) (void)hipHostFree(p); }
  } hf{hbuf};
  Leaves A, B;
  int64_t cur = 6, nwork = 6;
  Buf vs, vs_old, cntb, offb, bsum, ns, wk;  // ns: vertices made by the last split pass; wk: its new leaves
  uint64_t vcap = 1 << 16;
  if (prev) {
    // the seed from the previous grid's tree
    bool same = false;
    if (int rc = seed_from_grid(prev, P, cc, wp, A, wk, vs, &vcap, bsum, d_total, misc.as<uint32_t>() + 31,
                                d_vcount, hbuf, st, &cur, &nwork, prev->majorant_mode == o.majorant_mode, &same))
      return rc;
    if (same) {  // the previous tree is the result; its tets take the new volume's extinction
      hipLaunchKernelGGL(k_refresh_medium, dim3(nblocks(prev->n, 256)), dim3(256), 0, st, prev->n, prev->verts, P,
                         scale, o.majorant_mode, prev->rec, prev->rec32);
      TV_HIP(hipGetLastError());
      TV_HIP(hipEventRecord(e1, st));
      TV_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (unchanged_ms) *unchanged_ms = ms;  // *out stays NULL
      return TET_OK;
    }
    if (cur > o.max_tets) return fail(TET_ERR_CAPACITY, "leb_build: grid exceeds max_tets");
  } else {
    // roots
    const int64_t lcap = std::max<int64_t>(1 << 16, small ? small_cap : 0);
    if (!A.ensure(lcap) || !B.ensure(lcap)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: leaves");
    uint64_t hid[6], hv[24];
    const int p0[6] = {0, 0, 1, 1, 2, 2}, p1[6] = {1, 2, 0, 2, 0, 1};
    for (int r = 0; r < 6; r++) {
      int32_t c1[3] = {0, 0, 0}, c2[3] = {0, 0, 0};
      c1[p0[r]] = kLatS;
      c2[p0[r]] = kLatS;
      c2[p1[r]] = kLatS;
      hid[r] = 8 + r;
      hv[4 * r] = pack_vertex(0, 0, 0);
      hv[4 * r + 1] = pack_vertex(c1[0], c1[1], c1[2]);
      hv[4 * r + 2] = pack_vertex(c2[0], c2[1], c2[2]);
      hv[4 * r + 3] = pack_vertex(kLatS, kLatS, kLatS);
    }
    TV_HIP(hipMemcpyAsync(A.ids.p, hid, sizeof(hid), hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync(A.verts.p, hv, sizeof(hv), hipMemcpyHostToDevice, st));
    TV_HIP(hipMemsetAsync(A.flags.p, 0, 6, st));
    TV_HIP(hipMemsetAsync(A.chain.p, 0, 6 * 8, st));
    // the first worklist: the 6 roots
    if (!wk.ensure(small ? small_cap * 4 : 64)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: worklist");
    uint32_t w0[6] = {0, 1, 2, 3, 4, 5};
    TV_HIP(hipMemcpyAsync(wk.p, w0, sizeof(w0), hipMemcpyHostToDevice, st));
  }
  // vertex hash set
  // ns: the new-vertex set (nscap keys) followed by the cell map, both
  // cleared to all ones by one fill
  uint64_t nscap = 1024;
  if (!ns.ensure(nscap * 8 + kMapWords * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: new-vertex set");
  hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(nscap + kMapWords / 2, 256)), dim3(256), 0, st, ns.as<uint64_t>(),
                     (int64_t)(nscap + kMapWords / 2),
                     kEmptyKey);
  // capacities are even powers of two and grow by factors of 4, so the
  // sizes the set passes through do not depend on where it started (a
  // seed made its own set)
  if (!prev) {
    while (small && vcap < 4 * (uint64_t)small_cap) vcap <<= 2;  // stays at most half full in the small rounds
    if (!vs.ensure(vcap * 8)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: vertex set");
    hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(vcap, 256)), dim3(256), 0, st, vs.as<uint64_t>(), (int64_t)vcap,
                       kEmptyKey);
    hipLaunchKernelGGL(k_vset_seed, dim3(1), dim3(64), 0, st, A.verts.as<uint64_t>(), cur, vs.as<uint64_t>(),
                       vcap - 1, d_vcount);
  }
  int rounds = 0;
  bool done = false;
  int64_t nmain = -1;  // >= 0 once the tail rounds append (leaves below nmain stay in key order)
  bool dense_last = false;  // the last split pass kept no new-vertex set
  uint32_t splitc = 0;  // last value read of the running split count
  Buf anc;             // leaf below nmain each appended leaf descends from
  Buf cbox;            // tail rounds: cell box of every chunk of kChunk leaves
  if (small) {
    if (!cntb.ensure(small_cap * 4) || !bsum.ensure((size_t)small_blocks * 4))
      return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: counts");
    SmallRounds S;
    S.ids[0] = A.ids.as<uint64_t>();
    S.ids[1] = B.ids.as<uint64_t>();
    S.verts[0] = A.verts.as<uint64_t>();
    S.verts[1] = B.verts.as<uint64_t>();
    S.flags[0] = A.flags.as<uint8_t>();
    S.flags[1] = B.flags.as<uint8_t>();
    S.chain[0] = A.chain.as<uint64_t>();
    S.chain[1] = B.chain.as<uint64_t>();
    S.cnt = cntb.as<uint32_t>();
    S.bsum = bsum.as<uint32_t>();
    S.work = wk.as<uint32_t>();
    S.vset = vs.as<uint64_t>();
    S.vmask = vcap - 1;
    S.vcount = d_vcount;
    S.state = misc.as<uint32_t>() + 24;
    S.cur0 = cur;
    S.cap = small_cap;
    void* args[] = {&S, &P, &cc, &wp};
    // a refused cooperative launch (its blocks could not all be resident)
    // changed nothing: the host-driven rounds below then do all the work
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_small_rounds), dim3(small_blocks), dim3(256), args,
                                   0, st) != hipSuccess) {
      (void)hipGetLastError();
    } else {
      TV_HIP(hipMemcpyAsync(hbuf + 24, S.state, 24, hipMemcpyDeviceToHost, st));
      TV_HIP(hipStreamSynchronize(st));
      if (hbuf[29]) return fail(TET_ERR_INTERNAL, "leb_build: grid barrier of the small rounds timed out");
      cur = hbuf[24];
      rounds = (int)hbuf[25];
      nwork = 2 * (int64_t)hbuf[26];
      done = hbuf[27] != 0;
      if (rounds & 1) A.swap_with(B);
    }
  }
  while (!done) {
    if (!cntb.ensure(cur * 4) || !offb.ensure(cur * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: counts");
    if (nmain < 0)
      hipLaunchKernelGGL(k_mark, dim3(nblocks(cur, 256)), dim3(256), 0, st, cur, A.verts.as<uint64_t>(),
                         A.flags.as<uint8_t>(), cntb.as<uint32_t>(), vs.as<uint64_t>(), vcap - 1,
                         dense_last ? vs.as<uint64_t>() : ns.as<uint64_t>(), dense_last ? vcap - 1 : nscap - 1,
                         dense_last ? nullptr : (const uint32_t*)(ns.as<uint64_t>() + nscap), d_splitc, splitc,
                         nullptr);
    else
      hipLaunchKernelGGL(k_mark_tail, dim3(nblocks(cur, kChunk * kTailChunks)), dim3(kChunk), 0, st, cur, nmain,
                         A.verts.as<uint64_t>(), A.flags.as<uint8_t>(), vs.as<uint64_t>(), vcap - 1,
                         ns.as<uint64_t>(), nscap - 1, (const uint32_t*)(ns.as<uint64_t>() + nscap),
                         cbox.as<uint32_t>(), d_splitc, splitc, cntb.as<uint32_t>(), (int)(cur > nmain));
    if (nwork > 0)  // a seed from a previous grid may list no wanted leaf
      hipLaunchKernelGGL(k_want, dim3(nblocks(nwork, 256)), dim3(256), 0, st, nwork, wk.as<uint32_t>(),
                       A.ids.as<uint64_t>(), A.verts.as<uint64_t>(), A.flags.as<uint8_t>(), cntb.as<uint32_t>(), P,
                       cc, wp, vs.as<uint64_t>(), vcap - 1, d_splitc, splitc, nmain < 0 ? nullptr : cntb.as<uint32_t>());
    if (nmain < 0 && scan_u32(cntb.as<uint32_t>(), cur, offb.as<uint32_t>(), bsum, d_total, st))
      return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: scan");
    TV_HIP(hipMemcpyAsync(hbuf, d_total, (2 + kCountSlots) * 4, hipMemcpyDeviceToHost, st));
    TV_HIP(hipStreamSynchronize(st));
    const int64_t total = nmain < 0 ? (int64_t)hbuf[0] : cur + (int64_t)(hbuf[1] - splitc);
    uint64_t vcount = 0;
    for (int k = 0; k < kCountSlots; k++) vcount += hbuf[2 + k];
    splitc = hbuf[1];
    if (total == cur) break;
    rounds++;
    if (total > o.max_tets) return fail(TET_ERR_CAPACITY, "leb_build: grid exceeds max_tets");
    int64_t splits = total - cur;
    if ((vcount + (uint64_t)splits) * 2 > vcap) {  // keep the vertex set at most half full
      uint64_t ncap = vcap;
      while ((vcount + (uint64_t)splits) * 4 > ncap) ncap <<= 2;
      vs.swap_with(vs_old);
      if (!vs.ensure(ncap * 8)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: vertex set");
      hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(ncap, 256)), dim3(256), 0, st, vs.as<uint64_t>(), (int64_t)ncap,
                         kEmptyKey);
      TV_HIP(hipMemsetAsync(d_vcount, 0, kCountSlots * 4, st));
      hipLaunchKernelGGL(k_vset_rehash, dim3(nblocks(vcap, 256)), dim3(256), 0, st, vs_old.as<uint64_t>(),
                         (int64_t)vcap, vs.as<uint64_t>(), ncap - 1, d_vcount);
      vs_old.release();
      vcap = ncap;
    }
    const bool to_tail = nmain < 0 && splits * kAppendRatio < cur;  // the rounds after this one append
    if (nmain < 0) {
      if (!B.ensure(to_tail ? total + total / 16 : total)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: leaves");
    } else if (!A.grow_keep(total, cur, st) ||
               !grow_keep(anc, (size_t)(A.cap - nmain) * 4, (size_t)(cur - nmain) * 4, st)) {
      return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: leaves");
    }
    if (!wk.ensure((size_t)splits * 8)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: worklist");
    // A dense pass (more than leaves/8 splits: nearly every cell would be
    // marked) keeps no new-vertex set or cell map; the next round's checked
    // leaves probe the whole vertex set instead, which gives the same answer
    // (they can only have gained new vertices).  Otherwise: the new-vertex
    // set of this pass, at most half full, and its cell maps.
    const bool dense = nmain < 0 && splits * 8 > cur;
    dense_last = dense;
    if (!dense) {
      nscap = 1024;
      while ((uint64_t)splits * 2 > nscap) nscap <<= 1;
      if (!ns.ensure(nscap * 8 + kMapWords * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: new-vertex set");
      hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(nscap + kMapWords / 2, 256)), dim3(256), 0, st, ns.as<uint64_t>(),
                         (int64_t)(nscap + kMapWords / 2), kEmptyKey);
    }
    uint32_t* cells = (uint32_t*)(ns.as<uint64_t>() + nscap);
    if (nmain < 0) {
      hipLaunchKernelGGL(k_split, dim3(nblocks(cur, 256)), dim3(256), 0, st, cur, A.ids.as<uint64_t>(),
                         A.verts.as<uint64_t>(), A.flags.as<uint8_t>(), A.chain.as<uint64_t>(), cntb.as<uint32_t>(),
                         offb.as<uint32_t>(), B.ids.as<uint64_t>(), B.verts.as<uint64_t>(), B.flags.as<uint8_t>(),
                         B.chain.as<uint64_t>(), vs.as<uint64_t>(),
                         vcap - 1, d_vcount, dense ? nullptr : ns.as<uint64_t>(), nscap - 1, cells,
                         wk.as<uint32_t>());
      A.swap_with(B);
      // the tail: once few leaves split, the rounds after this one list the
      // splitting leaves and append children instead of compacting
      if (to_tail) {
        nmain = total;
        B.ids.release();
        B.verts.release();
        B.flags.release();
        B.chain.release();
        B.cap = 0;
        const int64_t chunks = nmain / kChunk;  // whole chunks of the main part
        if (!cbox.ensure((size_t)std::max<int64_t>(chunks, 1) * 32))
          return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: chunk boxes");
        if (chunks > 0)
          hipLaunchKernelGGL(k_chunk_boxes, dim3((unsigned)chunks), dim3(kChunk), 0, st, nmain, (int64_t)0, chunks,
                             A.verts.as<uint64_t>(), cbox.as<uint32_t>());
      }
    } else {
      hipLaunchKernelGGL(k_split_append, dim3(nblocks(splits, 256)), dim3(256), 0, st, splits, cntb.as<uint32_t>(),
                         cur, nmain, A.ids.as<uint64_t>(), A.verts.as<uint64_t>(), A.flags.as<uint8_t>(),
                         A.chain.as<uint64_t>(), anc.as<uint32_t>(), vs.as<uint64_t>(), vcap - 1, d_vcount,
                         ns.as<uint64_t>(), nscap - 1,
                         cells, wk.as<uint32_t>());
    }
    cur = total;
    nwork = 2 * splits;
  }
  vs.release();
  ns.release();
  wk.release();
  B.ids.release();
  B.verts.release();
  B.flags.release();
  B.chain.release();

  // finalize
  tet_grid* g = new tet_grid();
  memset(g, 0, sizeof(*g));
  TV_HIP(hipGetDevice(&g->device));
  g->n = cur;
  g->majorant_mode = o.majorant_mode;
  g->ids = (uint64_t*)dev_alloc(cur * 8);
  g->keys = (uint64_t*)dev_alloc(cur * 8);
  g->verts = (uint64_t*)dev_alloc(cur * 32);
  g->chain = (uint64_t*)dev_alloc(cur * 8);
  g->rec = (TetRec*)dev_alloc(cur * sizeof(TetRec));
  bool compact = o.majorant_mode == 0 && cur <= kMaxTets32;
  g->rec32 = compact ? (TetRec32*)dev_alloc(cur * sizeof(TetRec32)) : nullptr;
  if (!g->ids || !g->keys || !g->verts || !g->chain || !g->rec || (compact && !g->rec32)) {
    tet_grid_free(g);
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: grid arrays");
  }
  hipError_t he = hipSuccess;
  if (nmain < 0) {
    he = hipMemcpyAsync(g->ids, A.ids.p, cur * 8, hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(g->verts, A.verts.p, cur * 32, hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(g->chain, A.chain.p, cur * 8, hipMemcpyDeviceToDevice, st);
  } else {
    // depth-first order of the main part and the appended leaves
    const int64_t m = cur - nmain;
    Buf slots;
    if (!cntb.ensure(nmain * 4) || !offb.ensure(nmain * 4) || !slots.ensure(cur * 4)) {
      tet_grid_free(g);
      return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: merge");
    }
    uint32_t* gc = cntb.as<uint32_t>();
    uint32_t* pos = offb.as<uint32_t>();
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(nmain, 256)), dim3(256), 0, st, gc, nmain, 1u);
    hipLaunchKernelGGL(k_group_count, dim3(nblocks(m, 256)), dim3(256), 0, st, m, anc.as<uint32_t>(), gc);
    if (scan_u32(gc, nmain, pos, bsum, d_total, st)) {
      tet_grid_free(g);
      return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: merge");
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(nmain, 256)), dim3(256), 0, st, gc, nmain, 0u);
    hipLaunchKernelGGL(k_group_slots, dim3(nblocks(m, 256)), dim3(256), 0, st, m, anc.as<uint32_t>(), pos, gc,
                       slots.as<uint32_t>());
    hipLaunchKernelGGL(k_merge, dim3(nblocks(cur, 256)), dim3(256), 0, st, nmain, m, cur, A.ids.as<uint64_t>(),
                       A.verts.as<uint64_t>(), A.chain.as<uint64_t>(), anc.as<uint32_t>(), pos, slots.as<uint32_t>(),
                       g->ids, g->verts, g->chain);
    he = hipGetLastError();
    if (he == hipSuccess) he = hipStreamSynchronize(st);  // before the scratch returns to the pool
  }
  cntb.release();
  offb.release();
  bsum.release();
  anc.release();
  cbox.release();
  if (he == hipSuccess) {
    hipLaunchKernelGGL(k_keys, dim3(nblocks(cur, 1024)), dim3(1024), 0, st, cur, g->ids, g->keys, d_flag + 1);
    he = hipMemcpyAsync(&flag, d_flag + 1, 4, hipMemcpyDeviceToHost, st);
  }
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    tet_grid_free(g);
    return fail(TET_ERR_DEVICE, std::string("leb_build: ") + hipGetErrorString(he));
  }
  g->max_depth = flag;
  const uint32_t* shapes = shape_table();
  if (!shapes) {
    tet_grid_free(g);
    return fail(TET_ERR_DEVICE, "leb_build: shape table");
  }
  // bucket index of the keys: about 4 tets per bucket
  g->kbits = 4;
  while (g->kbits < 24 && (key_buckets(g->kbits + 1) << 2) <= cur) g->kbits++;
  g->kidx = (uint32_t*)dev_alloc((size_t)(key_buckets(g->kbits) + 1) * 4);
  if (!g->kidx) {
    tet_grid_free(g);
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: key index");
  }
  hipLaunchKernelGGL(k_key_index, dim3(nblocks(key_buckets(g->kbits) + 1, 256)), dim3(256), 0, st, cur, g->keys,
                     g->kbits, g->kidx);
  // records, then the links of the listed faces (at most 2 per tet in a
  // conforming grid)
  Buf items;
  const int64_t item_cap = 2 * cur + 64;
  if (!items.ensure((size_t)item_cap * 4)) {
    tet_grid_free(g);
    return fail(TET_ERR_OUT_OF_MEMORY, "leb_build: face list");
  }
  uint32_t* d_items = misc.as<uint32_t>() + 3;
  hipLaunchKernelGGL(k_records, dim3(nblocks(cur, kRecordsBlock)), dim3(kRecordsBlock), 0, st, cur, g->verts, P,
                     scale, o.majorant_mode, g->rec, g->rec32, items.as<uint32_t>(), item_cap, d_items,
                     d_flag + 2);
  hipLaunchKernelGGL(k_links, dim3(nblocks(item_cap, 128)), dim3(128), 0, st, items.as<uint32_t>(), d_items, item_cap,
                     cur, g->verts, g->keys, g->kidx, g->kbits, g->max_depth, shapes, g->rec, g->rec32, d_flag + 2);
  int ferr = 0;
  he = hipMemcpyAsync(&ferr, d_flag + 2, 4, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    tet_grid_free(g);
    return fail(TET_ERR_DEVICE, std::string("leb_build: ") + hipGetErrorString(he));
  }
  if (ferr) {
    tet_grid_free(g);
    return fail(TET_ERR_INTERNAL, "leb_build: grid failed the conformity check (code " + std::to_string(ferr) + ")");
  }
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g->stats.rounds = rounds;
  g->stats.max_depth = g->max_depth;
  g->stats.num_tets = cur;
  g->stats.ms = ms;
  *out = g;
  return TET_OK;
}

int build_grid(const tet_density* dens, const tet_camera* cam, float target_px, const tet_build_opts* opts_in,
               hipStream_t st, tet_grid** out) {
  if (out) *out = nullptr;
  if (!dens || !dens->data) return fail(TET_ERR_INVALID_ARG, "leb_build: density is NULL");
  return build_common(dens, nullptr, cam, target_px, opts_in, st, out);
}

int build_grid_sparse(const tet_sparse_density* sp, const tet_camera* cam, float target_px,
                      const tet_build_opts* opts_in, hipStream_t st, tet_grid** out) {
  if (out) *out = nullptr;
  if (!sp) return fail(TET_ERR_INVALID_ARG, "leb_build_sparse: density is NULL");
  return build_common(nullptr, sp, cam, target_px, opts_in, st, out);
}

// A rebuild for a new camera (or density, or options) seeded from the grid's
// current tree; the new arrays replace the old ones only on success (the
// grid's extra channels and density model, per tet, are dropped).  When the
// predicate keeps its value on every node of the tree, the grid is kept as
// it is (channels and model included).
static int update_common(tet_grid* g, const tet_density* dens, const tet_sparse_density* sp, const tet_camera* cam,
                         float target_px, const tet_build_opts* opts_in, hipStream_t st) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "leb_update: grid is NULL");
  int dev = -1;
  TV_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(TET_ERR_INVALID_ARG, "leb_update: the grid lives on another device");
  tet_grid* ng = nullptr;
  float same_ms = -1.0f;
  if (int rc = build_common(dens, sp, cam, target_px, opts_in, st, &ng, g, &same_ms)) return rc;
  if (!ng) {  // every node of the tree keeps its predicate: the grid is the result
    g->stats.rounds = 0;
    g->stats.ms = same_ms;
    return TET_OK;
  }
  std::swap(*g, *ng);
  tet_grid_free(ng);  // the previous arrays
  return TET_OK;
}

int update_grid(tet_grid* g, const tet_density* dens, const tet_camera* cam, float target_px,
                const tet_build_opts* opts_in, hipStream_t st) {
  if (!dens || !dens->data) return fail(TET_ERR_INVALID_ARG, "leb_update: density is NULL");
  return update_common(g, dens, nullptr, cam, target_px, opts_in, st);
}

int update_grid_sparse(tet_grid* g, const tet_sparse_density* sp, const tet_camera* cam, float target_px,
                       const tet_build_opts* opts_in, hipStream_t st) {
  if (!sp) return fail(TET_ERR_INVALID_ARG, "leb_update_sparse: density is NULL");
  return update_common(g, nullptr, sp, cam, target_px, opts_in, st);
}

// Extra channels: checked first (all of them), then reduced per tet; the
// grid's channels are replaced only when everything succeeded.
int grid_set_channels(tet_grid* g, const tet_channels* ch, hipStream_t st) {
  if (!g || !ch) return fail(TET_ERR_INVALID_ARG, "tet_grid_set_channels: NULL argument");
  const int32_t n = ch->n;
  if (n < 1 || n > 4096 || (n & (n - 1)))
    return fail(TET_ERR_INVALID_ARG, "tet_grid_set_channels: n must be a power of two <= 4096");
  int L = 0;
  while ((1 << L) < n) L++;
  const int64_t nvox = (int64_t)n * n * n;
  const float* src[3] = {ch->temperature, ch->albedo, ch->g};
  Buf copy[3], flag;
  const float* d[3] = {nullptr, nullptr, nullptr};
  if (!flag.ensure(4)) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_channels: scratch");
  TV_HIP(hipMemsetAsync(flag.p, 0, 4, st));
  for (int k = 0; k < 3; k++) {
    if (!src[k]) continue;
    d[k] = src[k];
    if (!ch->on_device) {
      if (!copy[k].ensure(nvox * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_channels: channel copy");
      TV_HIP(hipMemcpyAsync(copy[k].p, src[k], nvox * 4, hipMemcpyHostToDevice, st));
      d[k] = copy[k].as<float>();
    }
    hipLaunchKernelGGL(k_check_channel, dim3(nblocks(nvox, 256)), dim3(256), 0, st, d[k], nvox, k, flag.as<int>());
  }
  int bad = 0;
  TV_HIP(hipMemcpyAsync(&bad, flag.p, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  if (bad)
    return fail(TET_ERR_NUMERIC, "tet_grid_set_channels: temperature < 0 or not finite, albedo outside [0, 1] or g "
                                 "outside (-1, 1)");
  float* out[3] = {nullptr, nullptr, nullptr};
  struct Owned {
    float** o;
    bool keep = false;
    ~Owned() {
      if (!keep)
        for (int k = 0; k < 3; k++) dev_free(o[k]);
    }
  } own{out};
  for (int k = 0; k < 3; k++) {
    if (!d[k]) continue;
    out[k] = (float*)dev_alloc((size_t)g->n * 4);
    Pyramid P;
    std::vector<Buf> lv;
    if (!out[k] || !make_pyramid(d[k], n, L, P, lv, st))
      return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_channels: per-tet values");
    hipLaunchKernelGGL(k_channel_means, dim3(nblocks(g->n, 256)), dim3(256), 0, st, g->n, g->verts, P, out[k]);
    TV_HIP(hipGetLastError());
    TV_HIP(hipStreamSynchronize(st));  // before the pyramid returns to the pool
  }
  for (int k = 0; k < 3; k++) {
    dev_free(g->ch[k]);
    g->ch[k] = out[k];
  }
  own.keep = true;
  return TET_OK;
}

int grid_export_channels(const tet_grid* g, float* temperature, float* albedo, float* gch, int32_t on_device) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_channels: grid is NULL");
  float* dst[3] = {temperature, albedo, gch};
  for (int k = 0; k < 3; k++)
    if (dst[k] && !g->ch[k]) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_channels: the grid has no such channel");
  for (int k = 0; k < 3; k++)
    if (dst[k])
      TV_HIP(hipMemcpy(dst[k], g->ch[k], (size_t)g->n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return TET_OK;
}

// ---------------------------------------------------------------- density models
// Trilinear sample (FP64, unscaled) of the volume at lattice point (x, y, z):
// voxel-centre coordinates u = v n / 2^20 - 1/2, indices clamped to the
// volume, interpolated along x, then y, then z.
__device__ inline double trilinear_at(const float* __restrict__ d, int32_t n, const int64_t p[3]) {
  int64_t i0[3], i1[3];
  double f[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double u = (double)p[a] * (double)n / (double)kLatS - 0.5;
    const double fl = floor(u);
    f[a] = u - fl;
    const int64_t lo = (int64_t)fl, hi = lo + 1;
    i0[a] = lo < 0 ? 0 : (lo > n - 1 ? n - 1 : lo);
    i1[a] = hi < 0 ? 0 : (hi > n - 1 ? n - 1 : hi);
  }
  double cz[2];
#pragma unroll
  for (int c = 0; c < 2; c++) {
    const int64_t z = c ? i1[2] : i0[2];
    double cy[2];
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int64_t y = b ? i1[1] : i0[1];
      const double d0 = (double)d[i0[0] + (int64_t)n * (y + (int64_t)n * z)];
      const double d1 = (double)d[i1[0] + (int64_t)n * (y + (int64_t)n * z)];
      cy[b] = (1.0 - f[0]) * d0 + f[0] * d1;
    }
    cz[c] = (1.0 - f[1]) * cy[0] + f[1] * cy[1];
  }
  return (1.0 - f[2]) * cz[0] + f[2] * cz[1];
}

// Model 1 (one thread per tet): vertex values rho_j = scale * trilinear
// sample; majorant = max rho_j; the affine function through them, gradient
// by Cramer's rule on the lattice edge vectors e_k = v_k - v_0 (cross
// products and determinant exact in int64), g = (dr_1 (e_2 x e_3) + dr_2
// (e_3 x e_1) + dr_3 (e_1 x e_2)) / det * 2^20 (world units), c0 = rho_0 -
// g . v_0; FP64, rounded to FP32.
__global__ void k_model_linear(int64_t n, const uint64_t* __restrict__ verts, const float* __restrict__ d,
                               int32_t nv, double scale, float* __restrict__ maj, float4* __restrict__ coef) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int64_t v[4][3];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const uint64_t pv = verts[4 * t + j];
    v[j][0] = vx(pv);
    v[j][1] = vy(pv);
    v[j][2] = vz(pv);
  }
  double rho[4], mx = 0.0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    rho[j] = scale * trilinear_at(d, nv, v[j]);
    if (j == 0 || rho[j] > mx) mx = rho[j];
  }
  int64_t e[3][3], c[3][3];
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int a = 0; a < 3; a++) e[k][a] = v[k + 1][a] - v[0][a];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const int64_t* p = e[(k + 1) % 3];
    const int64_t* q = e[(k + 2) % 3];
    c[k][0] = p[1] * q[2] - p[2] * q[1];
    c[k][1] = p[2] * q[0] - p[0] * q[2];
    c[k][2] = p[0] * q[1] - p[1] * q[0];
  }
  const int64_t det = e[0][0] * c[0][0] + e[0][1] * c[0][1] + e[0][2] * c[0][2];
  const double dr[3] = {rho[1] - rho[0], rho[2] - rho[0], rho[3] - rho[0]};
  double g[3];
#pragma unroll
  for (int a = 0; a < 3; a++)
    g[a] = ((dr[0] * (double)c[0][a] + dr[1] * (double)c[1][a]) + dr[2] * (double)c[2][a]) / (double)det *
           (double)kLatS;
  const double p0[3] = {(double)v[0][0] / kLatS, (double)v[0][1] / kLatS, (double)v[0][2] / kLatS};
  const double c0 = rho[0] - ((g[0] * p0[0] + g[1] * p0[1]) + g[2] * p0[2]);
  maj[t] = (float)mx;
  coef[t] = make_float4((float)c0, (float)g[0], (float)g[1], (float)g[2]);
}

// Model 2 (one thread per tet): majorant = scale * the largest voxel of the
// tet's open bounding box (the pyramid's exact maxima).
__global__ void k_model_voxel(int64_t n, const uint64_t* __restrict__ verts, Pyramid P, double scale,
                              float* __restrict__ maj) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t v[4] = {verts[4 * t], verts[4 * t + 1], verts[4 * t + 2], verts[4 * t + 3]};
  int32_t lo[3], hi[3];
  tet_box(v, lo, hi);
  float mn, mx;
  double s, c;
  box_stats(P, lo, hi, mn, mx, s, c);
  maj[t] = (float)(scale * (double)mx);
}

// Model records: the grid's records with the model's majorant as the
// extinction (and majorant) every walk step reads.
__global__ void k_model_records(int64_t n, const TetRec* __restrict__ rec, const TetRec32* __restrict__ rec32,
                                const float* __restrict__ maj, TetRec* __restrict__ mrec, TetRec32* __restrict__ mrec32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float m = maj[t];
  TetRec r = rec[t];
  r.sigma = m;
  r.majorant = m;
  mrec[t] = r;
  if (rec32) {
    TetRec32 q = rec32[t];
    q.w[3] = __float_as_uint(m);
    mrec32[t] = q;
  }
}

// Checked first (the grid is unchanged on any error), then built whole and
// swapped in.
int grid_set_density_model(tet_grid* g, const tet_density* dens, int32_t model, hipStream_t st) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_grid_set_density_model: grid is NULL");
  if (model < 0 || model > 2) return fail(TET_ERR_INVALID_ARG, "tet_grid_set_density_model: model must be 0, 1 or 2");
  auto drop = [&]() {
    dev_free(g->mmaj);
    dev_free(g->mcoef);
    dev_free(g->mdens);
    dev_free(g->mrec);
    dev_free(g->mrec32);
    g->mmaj = nullptr;
    g->mcoef = nullptr;
    g->mdens = nullptr;
    g->mrec = nullptr;
    g->mrec32 = nullptr;
    g->model = 0;
  };
  if (model == 0) {
    drop();
    return TET_OK;
  }
  if (!dens || !dens->data) return fail(TET_ERR_INVALID_ARG, "tet_grid_set_density_model: no volume");
  const int32_t n = dens->n;
  if (n < 1 || n > 4096 || (n & (n - 1)))
    return fail(TET_ERR_INVALID_ARG, "tet_grid_set_density_model: n must be a power of two <= 4096");
  if (!(dens->density_scale > 0.0f) || std::isinf(dens->density_scale))
    return fail(TET_ERR_INVALID_ARG, "tet_grid_set_density_model: density_scale must be finite and > 0");
  int L = 0;
  while ((1 << L) < n) L++;
  const int64_t nvox = (int64_t)n * n * n;
  // the volume on the device: the model's own copy for voxel lookups, else
  // a temporary one for host input
  float* vol = nullptr;
  Buf tmp, flag;
  const float* d = dens->data;
  if (model == 2) {
    vol = (float*)dev_alloc((size_t)nvox * 4);
    if (!vol) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_density_model: volume copy");
    TV_HIP(hipMemcpyAsync(vol, d, (size_t)nvox * 4, dens->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          st));
    d = vol;
  } else if (!dens->on_device) {
    if (!tmp.ensure((size_t)nvox * 4)) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_density_model: volume copy");
    TV_HIP(hipMemcpyAsync(tmp.p, d, (size_t)nvox * 4, hipMemcpyHostToDevice, st));
    d = tmp.as<float>();
  }
  struct Owned {
    float* vol;
    float* maj = nullptr;
    float4* coef = nullptr;
    TetRec* rec = nullptr;
    TetRec32* rec32 = nullptr;
    bool keep = false;
    ~Owned() {
      if (keep) return;
      dev_free(vol);
      dev_free(maj);
      dev_free(coef);
      dev_free(rec);
      dev_free(rec32);
    }
  } own{vol};
  if (!flag.ensure(4)) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_density_model: scratch");
  TV_HIP(hipMemsetAsync(flag.p, 0, 4, st));
  hipLaunchKernelGGL(k_check_density, dim3(nblocks(nvox, 256)), dim3(256), 0, st, d, nvox, flag.as<int>());
  int bad = 0;
  TV_HIP(hipMemcpyAsync(&bad, flag.p, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  if (bad) return fail(TET_ERR_NUMERIC, "tet_grid_set_density_model: density values must be finite and >= 0");
  own.maj = (float*)dev_alloc((size_t)g->n * 4);
  own.rec = (TetRec*)dev_alloc((size_t)g->n * sizeof(TetRec));
  if (g->rec32) own.rec32 = (TetRec32*)dev_alloc((size_t)g->n * sizeof(TetRec32));
  if (model == 1) own.coef = (float4*)dev_alloc((size_t)g->n * sizeof(float4));
  if (!own.maj || !own.rec || (g->rec32 && !own.rec32) || (model == 1 && !own.coef))
    return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_density_model: per-tet model");
  const unsigned blocks = nblocks(g->n, 256);
  if (model == 1) {
    hipLaunchKernelGGL(k_model_linear, dim3(blocks), dim3(256), 0, st, g->n, g->verts, d, n,
                       (double)dens->density_scale, own.maj, own.coef);
    TV_HIP(hipGetLastError());
  } else {
    Pyramid P;
    std::vector<Buf> lv;
    if (!make_pyramid(d, n, L, P, lv, st)) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_set_density_model: pyramid");
    hipLaunchKernelGGL(k_model_voxel, dim3(blocks), dim3(256), 0, st, g->n, g->verts, P, (double)dens->density_scale,
                       own.maj);
    TV_HIP(hipGetLastError());
    TV_HIP(hipStreamSynchronize(st));  // before the pyramid returns to the pool
  }
  hipLaunchKernelGGL(k_model_records, dim3(blocks), dim3(256), 0, st, g->n, g->rec, g->rec32, own.maj, own.rec,
                     own.rec32);
  TV_HIP(hipGetLastError());
  TV_HIP(hipStreamSynchronize(st));
  drop();
  g->mmaj = own.maj;
  g->mcoef = own.coef;
  g->mdens = own.vol;
  g->mrec = own.rec;
  g->mrec32 = own.rec32;
  g->mn = n;
  g->mscale = dens->density_scale;
  g->model = model;
  own.keep = true;
  return TET_OK;
}

int grid_export_density_model(const tet_grid* g, float* majorant, float* coef, int32_t on_device) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_density_model: grid is NULL");
  if (g->model == 0) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_density_model: the grid has no density model");
  if (coef && g->model != 1)
    return fail(TET_ERR_INVALID_ARG, "tet_grid_export_density_model: coefficients exist for the linear model only");
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (majorant) TV_HIP(hipMemcpy(majorant, g->mmaj, (size_t)g->n * 4, kind));
  if (coef) TV_HIP(hipMemcpy(coef, g->mcoef, (size_t)g->n * 16, kind));
  return TET_OK;
}

}  // namespace tv
