/*
 * leb.c -- plain CPU statement of the grid construction ("Grid Construction"
 * section of the paper).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * What is computed, in the paper's order:
 *   1. Roots.  The paper tessellates the control cube into 24 tets, one per
 *      half-edge of the cube (vertices: the half-edge's endpoints, the centre
 *      of the face carrying it, the cube centre).  Reading: those 24 tets are
 *      exactly the depth-2 descendants of the 6 Kuhn tets of the cube under
 *      Maubach bisection, so the roots here are the 6 Kuhn tets and "paper
 *      depth d" is depth d + 2 here.  (Pinned by a test.)
 *   2. Bisection after Maubach (1995): a tet (x0,x1,x2,x3) at depth d has tag
 *      k = 3 - (d mod 3); its refinement edge is (x0, xk), which is the
 *      unique longest edge of every tet of these grids (pinned by a test);
 *      children:  first  = (x0..x_{k-1}, z, x_{k+1}..x3),
 *                 second = (x1..x_k,     z, x_{k+1}..x3),  z = (x0+xk)/2.
 *   3. Propagation (the paper spreads each bisection to the neighbours by a
 *      fixed rule that keeps the grid conforming).  Reading: the recursive conforming refinement of a tet T:
 *      while some leaf sharing T's refinement edge e has a different
 *      refinement edge, refine that leaf first; then bisect every leaf of the
 *      star of e.  This keeps the mesh conforming after every call.
 *   4. Subdivision criteria.  Density variation: (max D - min D) / mean D
 *      above a threshold tau.  Reading of D (the paper: every density value
 *      inside the cell): the voxels overlapping the open bounding box of the
 *      tet, summarised through a min/max/sum pyramid (definition below).
 *      Camera: no split outside the view frustum or below a projected size
 *      of target_px pixels.  Reading of both tests: see want_camera().
 *   5. Neighbour table: for each face, the unique other leaf having the same
 *      three vertices (found by hashing sorted vertex triples), plus the
 *      index of that face in the neighbour ("back face").
 *   6. Per-tet medium: one extinction value per tet (the paper stores one
 *      density per tet).  Reading: density_scale * mean(D(T)); the
 *      majorant is that value (tight) or density_scale * max(D(T)).
 *   7. Face orientation codes: the outward normal of every face is one of 18
 *      directions (+-axes, +-face diagonals); code = 2 * (direction index) +
 *      sign, with the plane offset n_f . v in lattice units.
 *   8. Extra channels (the paper's implementation also carries e.g.
 *      temperature, albedo and phase-function parameters per tet).  Reading:
 *      each channel given on its own n^3 voxel grid is reduced per tet like
 *      the density, to the mean over the voxels of the tet's box (same box
 *      rule and summation order), stored FP32.
 *   9. Density inside a tet (an extension: the paper keeps one value per
 *      tet).  Model 1, linear: the density is sampled at each vertex by
 *      trilinear interpolation of the volume (values at voxel centres
 *      (i + 1/2) / n, indices clamped at the cube's faces; FP64, x then y
 *      then z), times the scale, and interpolated linearly inside the tet;
 *      the majorant is the largest vertex value, which bounds a linear
 *      function on the tet.  Model 2, voxel lookup: the extinction at a
 *      point is the scale times the voxel containing it; the majorant is
 *      the scale times the largest voxel of the tet's box (the rule of
 *      item 4; every interior point lies in that box).  Both make the null
 *      collisions of delta tracking real ones rather than no-ops.
 *
 * Coordinates: world = unit cube; lattice = world * 2^20 (integers, exact).
 * Heap ids: roots 8..13; children of h are 2h and 2h+1; depth = bits - 4.
 * Canonical tet order: depth-first key id << (60 - depth), ascending.
 */
#include "oracle_internal.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

const int32_t or_dirs[9][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

/* Axis orders of the 6 Kuhn roots. */
static const int kuhn_perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                    {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

uint64_t or_mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

static int depth_of_id(uint64_t id) {
  int b = 0;
  while ((id >> b) > 1) b++;
  return b - 3; /* roots 8..13 have 4 bits -> depth 0 */
}

static uint64_t dfs_key(uint64_t id) { return id << (60 - depth_of_id(id)); }

static uint64_t vkey(const int32_t* p) {
  return (uint64_t)p[0] | ((uint64_t)p[1] << 21) | ((uint64_t)p[2] << 42);
}

/* ------------------------------------------------------------------ */
/* Node storage                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t id;
  int32_t v[4][3];
  int32_t depth;
  uint8_t alive;   /* 1 = current leaf */
  uint8_t checked; /* want() already evaluated (it depends on the tet only) */
} onode;

#define EDGE_CAP 16
typedef struct {
  uint64_t a, b;
  int32_t used, cnt;
  int32_t m[EDGE_CAP];
} edge_ent;

typedef struct {
  /* inputs */
  const float* dens;
  int32_t n, L; /* n = 2^L voxels per axis */
  ocam cam;
  obuild_opts o;
  /* pyramid levels 1..L: min, max, FP64 sum; level 0 = the voxels */
  float** pmn;
  float** pmx;
  double** psum;
  /* camera frame, FP64 */
  double pos[3], f[3], side[4][3], kpx2, tgt2;
  /* nodes */
  onode* nd;
  int64_t nn, ncap, nleaves;
  /* edge -> leaves having that edge */
  edge_ent* et;
  uint64_t ecap, ecount;
  int err;
} bctx;

static int64_t new_node(bctx* c) {
  if (c->nn == c->ncap) {
    int64_t nc = c->ncap ? c->ncap * 2 : 1024;
    onode* p = (onode*)realloc(c->nd, (size_t)nc * sizeof(onode));
    if (!p) { c->err = -2; return -1; }
    c->nd = p;
    c->ncap = nc;
  }
  memset(&c->nd[c->nn], 0, sizeof(onode));
  return c->nn++;
}

/* ---------------- edge map ---------------- */
static uint64_t edge_hash(uint64_t a, uint64_t b) { return or_mix64(a * 0x9E3779B97F4A7C15ull ^ or_mix64(b)); }

static edge_ent* edge_find(bctx* c, uint64_t a, uint64_t b, int create);

static int edge_grow(bctx* c) {
  uint64_t oc = c->ecap;
  edge_ent* old = c->et;
  uint64_t nc = oc ? oc * 2 : (1u << 16);
  c->et = (edge_ent*)calloc((size_t)nc, sizeof(edge_ent));
  if (!c->et) { c->et = old; c->err = -2; return -1; }
  c->ecap = nc;
  c->ecount = 0;
  for (uint64_t i = 0; i < oc; i++) {
    if (old[i].used && old[i].cnt > 0) {
      edge_ent* e = edge_find(c, old[i].a, old[i].b, 1);
      e->cnt = old[i].cnt;
      memcpy(e->m, old[i].m, sizeof(e->m));
    }
  }
  free(old);
  return 0;
}

static edge_ent* edge_find(bctx* c, uint64_t a, uint64_t b, int create) {
  if (a > b) { uint64_t t = a; a = b; b = t; }
  if (create && (c->ecount + 1) * 2 > c->ecap) {
    if (edge_grow(c)) return NULL;
  }
  if (!c->ecap) return NULL;
  uint64_t i = edge_hash(a, b) & (c->ecap - 1);
  for (;;) {
    edge_ent* e = &c->et[i];
    if (!e->used) {
      if (!create) return NULL;
      e->used = 1;
      e->a = a;
      e->b = b;
      e->cnt = 0;
      c->ecount++;
      return e;
    }
    if (e->a == a && e->b == b) return e;
    i = (i + 1) & (c->ecap - 1);
  }
}

static void edges_of(const onode* t, uint64_t ea[6], uint64_t eb[6]) {
  int q = 0;
  for (int i = 0; i < 4; i++)
    for (int j = i + 1; j < 4; j++) {
      ea[q] = vkey(t->v[i]);
      eb[q] = vkey(t->v[j]);
      q++;
    }
}

static void edge_attach(bctx* c, int64_t ti) {
  uint64_t ea[6], eb[6];
  edges_of(&c->nd[ti], ea, eb);
  for (int q = 0; q < 6; q++) {
    edge_ent* e = edge_find(c, ea[q], eb[q], 1);
    if (!e) return;
    if (e->cnt >= EDGE_CAP) { c->err = -7; return; }
    e->m[e->cnt++] = (int32_t)ti;
  }
}

static void edge_detach(bctx* c, int64_t ti) {
  uint64_t ea[6], eb[6];
  edges_of(&c->nd[ti], ea, eb);
  for (int q = 0; q < 6; q++) {
    edge_ent* e = edge_find(c, ea[q], eb[q], 0);
    if (!e) { c->err = -7; return; }
    int w = 0;
    for (int r = 0; r < e->cnt; r++)
      if (e->m[r] != (int32_t)ti) e->m[w++] = e->m[r];
    e->cnt = w;
  }
}

/* ---------------- Maubach bisection ---------------- */
static int tag_of(int depth) { return 3 - (depth % 3); }

static void refinement_edge(const onode* t, uint64_t* a, uint64_t* b) {
  int k = tag_of(t->depth);
  uint64_t p = vkey(t->v[0]), q = vkey(t->v[k]);
  *a = p < q ? p : q;
  *b = p < q ? q : p;
}

static void bisect(bctx* c, int64_t ti) {
  int64_t c1 = new_node(c);
  int64_t c2 = new_node(c);
  if (c1 < 0 || c2 < 0) return;
  onode* t = &c->nd[ti];
  onode* a = &c->nd[c1];
  onode* b = &c->nd[c2];
  int k = tag_of(t->depth);
  int32_t z[3];
  for (int i = 0; i < 3; i++) {
    int32_t s = t->v[0][i] + t->v[k][i];
    if (s & 1) { c->err = -7; return; } /* beyond lattice resolution */
    z[i] = s / 2;
  }
  /* first child: x_k replaced by z */
  for (int j = 0; j < 4; j++) memcpy(a->v[j], t->v[j], sizeof(z));
  memcpy(a->v[k], z, sizeof(z));
  /* second child: (x1..x_k, z, x_{k+1}..x3) */
  for (int j = 0; j < k; j++) memcpy(b->v[j], t->v[j + 1], sizeof(z));
  memcpy(b->v[k], z, sizeof(z));
  for (int j = k + 1; j < 4; j++) memcpy(b->v[j], t->v[j], sizeof(z));
  a->id = 2 * t->id;
  b->id = 2 * t->id + 1;
  a->depth = b->depth = t->depth + 1;
  a->alive = b->alive = 1;
  edge_detach(c, ti);
  t->alive = 0;
  edge_attach(c, c1);
  edge_attach(c, c2);
  c->nleaves += 1;
}

/* Conforming refinement of leaf ti (recursive closure). */
static void refine(bctx* c, int64_t ti, int level) {
  if (c->err || !c->nd[ti].alive) return;
  if (level > 4096) { c->err = -7; return; }
  uint64_t ea, eb;
  refinement_edge(&c->nd[ti], &ea, &eb);
  for (;;) {
    edge_ent* e = edge_find(c, ea, eb, 0);
    if (!e) { c->err = -7; return; }
    int64_t bad = -1;
    for (int r = 0; r < e->cnt; r++) {
      uint64_t xa, xb;
      refinement_edge(&c->nd[e->m[r]], &xa, &xb);
      if (xa != ea || xb != eb) { bad = e->m[r]; break; }
    }
    if (bad < 0) break;
    refine(c, bad, level + 1);
    if (c->err) return;
    if (!c->nd[ti].alive) return;
  }
  edge_ent* e = edge_find(c, ea, eb, 0);
  int32_t star[EDGE_CAP];
  int ns = e->cnt;
  memcpy(star, e->m, sizeof(int32_t) * (size_t)ns);
  for (int r = 0; r < ns; r++) {
    bisect(c, star[r]);
    if (c->err) return;
  }
}

/* ------------------------------------------------------------------ */
/* Density pyramid and statistics D(T)                                  */
/* ------------------------------------------------------------------ */
/* Level l >= 1 cell (i,j,k) covers the 2^l voxels per axis starting at
 * (i,j,k) * 2^l.  min / max are exact; the sum is FP64 with the eight
 * children (a,b,c) = x,y,z offsets combined as
 *   ((c000 + c100) + (c010 + c110)) + ((c001 + c101) + (c011 + c111)).   */
static float lv_min(const bctx* c, int l, int64_t idx) { return l == 0 ? c->dens[idx] : c->pmn[l][idx]; }
static float lv_max(const bctx* c, int l, int64_t idx) { return l == 0 ? c->dens[idx] : c->pmx[l][idx]; }
static double lv_sum(const bctx* c, int l, int64_t idx) { return l == 0 ? (double)c->dens[idx] : c->psum[l][idx]; }

static int build_pyramid(bctx* c) {
  int L = c->L;
  c->pmn = (float**)calloc((size_t)L + 1, sizeof(float*));
  c->pmx = (float**)calloc((size_t)L + 1, sizeof(float*));
  c->psum = (double**)calloc((size_t)L + 1, sizeof(double*));
  if (!c->pmn || !c->pmx || !c->psum) return -2;
  for (int l = 1; l <= L; l++) {
    int64_t m = (int64_t)c->n >> l, pm = (int64_t)c->n >> (l - 1);
    size_t cnt = (size_t)(m * m * m);
    c->pmn[l] = (float*)malloc(cnt * sizeof(float));
    c->pmx[l] = (float*)malloc(cnt * sizeof(float));
    c->psum[l] = (double*)malloc(cnt * sizeof(double));
    if (!c->pmn[l] || !c->pmx[l] || !c->psum[l]) return -2;
    for (int64_t k = 0; k < m; k++)
      for (int64_t j = 0; j < m; j++)
        for (int64_t i = 0; i < m; i++) {
          int64_t ch[8];
          for (int q = 0; q < 8; q++) {
            int64_t a = q & 1, b = (q >> 1) & 1, cc = (q >> 2) & 1;
            ch[q] = (2 * i + a) + pm * ((2 * j + b) + pm * (2 * k + cc));
          }
          float mn = lv_min(c, l - 1, ch[0]), mx = lv_max(c, l - 1, ch[0]);
          for (int q = 1; q < 8; q++) {
            float a = lv_min(c, l - 1, ch[q]), b = lv_max(c, l - 1, ch[q]);
            if (a < mn) mn = a;
            if (b > mx) mx = b;
          }
          double s = ((lv_sum(c, l - 1, ch[0]) + lv_sum(c, l - 1, ch[1])) +
                      (lv_sum(c, l - 1, ch[2]) + lv_sum(c, l - 1, ch[3]))) +
                     ((lv_sum(c, l - 1, ch[4]) + lv_sum(c, l - 1, ch[5])) +
                      (lv_sum(c, l - 1, ch[6]) + lv_sum(c, l - 1, ch[7])));
          int64_t o = i + m * (j + m * k);
          c->pmn[l][o] = mn;
          c->pmx[l][o] = mx;
          c->psum[l][o] = s;
        }
  }
  return 0;
}

static void free_pyramid(bctx* c) {
  if (c->pmn)
    for (int l = 1; l <= c->L; l++) { free(c->pmn[l]); free(c->pmx[l]); free(c->psum[l]); }
  free(c->pmn);
  free(c->pmx);
  free(c->psum);
  c->pmn = c->pmx = NULL;
  c->psum = NULL;
}

/* D(box): voxels overlapping the open lattice box (lo, hi).  Their index
 * range per axis is [floor(lo/vs), ceil(hi/vs) - 1] (vs = voxel size).  The
 * range is summarised at the coarsest pyramid level l at which every range
 * start and end+1 is a multiple of 2^l; the cells are combined in ascending
 * z, then y, then x order, sum accumulated left to right from 0.0. */
static void box_stats(const bctx* c, const int32_t lo[3], const int32_t hi[3], float* mn, float* mx,
                      double* sum, double* count) {
  int64_t vs = (int64_t)OR_LAT_S / c->n;
  int64_t r0[3], r1[3];
  for (int a = 0; a < 3; a++) {
    r0[a] = lo[a] / vs;
    r1[a] = (hi[a] + vs - 1) / vs; /* one past the last voxel */
  }
  int l = c->L;
  for (; l > 0; l--) {
    int ok = 1;
    for (int a = 0; a < 3; a++)
      if ((r0[a] % ((int64_t)1 << l)) != 0 || (r1[a] % ((int64_t)1 << l)) != 0) ok = 0;
    if (ok) break;
  }
  int64_t m = (int64_t)c->n >> l;
  double s = 0.0;
  float lo_v = 0, hi_v = 0;
  int first = 1;
  int64_t cells = 0;
  for (int64_t k = r0[2] >> l; k < r1[2] >> l; k++)
    for (int64_t j = r0[1] >> l; j < r1[1] >> l; j++)
      for (int64_t i = r0[0] >> l; i < r1[0] >> l; i++) {
        int64_t o = i + m * (j + m * k);
        float a = lv_min(c, l, o), b = lv_max(c, l, o);
        if (first || a < lo_v) lo_v = a;
        if (first || b > hi_v) hi_v = b;
        first = 0;
        s = s + lv_sum(c, l, o);
        cells++;
      }
  *mn = lo_v;
  *mx = hi_v;
  *sum = s;
  *count = (double)cells * (double)((int64_t)1 << (3 * l));
}

static void tet_box(const int32_t v[4][3], int32_t lo[3], int32_t hi[3]) {
  for (int a = 0; a < 3; a++) {
    lo[a] = hi[a] = v[0][a];
    for (int j = 1; j < 4; j++) {
      if (v[j][a] < lo[a]) lo[a] = v[j][a];
      if (v[j][a] > hi[a]) hi[a] = v[j][a];
    }
  }
}

/* ------------------------------------------------------------------ */
/* Subdivision criteria                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static void normalize3(double* v) {
  double l = sqrt(dot3(v, v));
  v[0] = v[0] / l;
  v[1] = v[1] / l;
  v[2] = v[2] / l;
}

static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Camera frame in FP64 from the FP32 camera. */
static void camera_frame(bctx* c) {
  const ocam* k = &c->cam;
  double look[3], up[3], r[3], u[3];
  for (int i = 0; i < 3; i++) {
    c->pos[i] = (double)k->pos[i];
    look[i] = (double)k->look_at[i];
    up[i] = (double)k->up[i];
    c->f[i] = look[i] - c->pos[i];
  }
  normalize3(c->f);
  cross3(c->f, up, r);
  normalize3(r);
  cross3(r, c->f, u);
  double tan_y = tan((double)k->fov_y_deg * (3.14159265358979323846 / 360.0));
  double tan_x = tan_y * (double)k->width / (double)k->height;
  double kpx = ((double)k->height * 0.5) / tan_y;
  for (int i = 0; i < 3; i++) {
    c->side[0][i] = tan_x * c->f[i] - r[i];
    c->side[1][i] = tan_x * c->f[i] + r[i];
    c->side[2][i] = tan_y * c->f[i] - u[i];
    c->side[3][i] = tan_y * c->f[i] + u[i];
  }
  for (int p = 0; p < 4; p++) normalize3(c->side[p]);
  c->kpx2 = kpx * kpx;
  c->tgt2 = (double)c->o.target_px * (double)c->o.target_px;
}

/* Camera criterion.  Reading (the paper gives no measure of a tet's projected
 * size against one pixel): centroid c, bounding radius l = longest edge
 * (>= 4/3 of the largest centroid-vertex distance), w = c - pos.
 *   in frustum  <=>  f.w >= -l and n_p.w >= -l for the 4 inward side normals
 *   big enough  <=>  |w|^2 <= l^2  or  l^2 k_px^2 > target^2 |w|^2
 * with k_px = (H/2) / tan(fov_y / 2).  All FP64 from exact inputs. */
static int want_camera(const bctx* c, const int32_t v[4][3], int depth) {
  int k = tag_of(depth);
  double cw[3], w[3];
  for (int i = 0; i < 3; i++) {
    int64_t s = (int64_t)v[0][i] + v[1][i] + v[2][i] + v[3][i];
    cw[i] = (double)s * 0x1p-22;
    w[i] = cw[i] - c->pos[i];
  }
  int64_t l2i = 0;
  for (int i = 0; i < 3; i++) {
    int64_t e = (int64_t)v[k][i] - v[0][i];
    l2i += e * e;
  }
  double l2 = (double)l2i * 0x1p-40;
  double l = sqrt(l2);
  if (dot3(c->f, w) < -l) return 0;
  for (int p = 0; p < 4; p++)
    if (dot3(c->side[p], w) < -l) return 0;
  double z2 = dot3(w, w);
  if (z2 <= l2) return 1;
  return l2 * c->kpx2 > c->tgt2 * z2;
}

/* Density-variation criterion: (max D - min D) > tau * mean D, mean > 0. */
static int want_variation(const bctx* c, const int32_t v[4][3]) {
  int32_t lo[3], hi[3];
  float mn, mx;
  double s, cnt;
  tet_box(v, lo, hi);
  box_stats(c, lo, hi, &mn, &mx, &s, &cnt);
  double mean = s / cnt;
  if (!(mean > 0.0)) return 0;
  return ((double)mx - (double)mn) > c->o.variation_tau * mean;
}

static int want(const bctx* c, const int32_t v[4][3], int depth, uint64_t id) {
  switch (c->o.want_mode) {
    case 1:
      return depth < c->o.uniform_depth;
    case 2:
      return depth < c->o.max_depth && (int32_t)(or_mix64(id ^ c->o.rand_seed) & 0xFFFF) < c->o.rand_thresh;
    default:
      if (depth >= c->o.max_depth) return 0;
      if (!want_variation(c, v)) return 0;
      return want_camera(c, v, depth);
  }
}

/* ------------------------------------------------------------------ */
/* Faces, neighbours, medium                                            */
/* ------------------------------------------------------------------ */
/* Outward unit normal (entries in {-1,0,1}) and orientation code of face f
 * (the face opposite vertex f). */
static int face_code(const int32_t v[4][3], int f, int32_t un[3], int32_t* off) {
  int idx[3], q = 0;
  for (int j = 0; j < 4; j++)
    if (j != f) idx[q++] = j;
  int64_t e1[3], e2[3], n[3], w[3];
  for (int i = 0; i < 3; i++) {
    e1[i] = (int64_t)v[idx[1]][i] - v[idx[0]][i];
    e2[i] = (int64_t)v[idx[2]][i] - v[idx[0]][i];
    w[i] = (int64_t)v[f][i] - v[idx[0]][i];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  int64_t s = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
  if (s == 0) return -1;
  if (s > 0)
    for (int i = 0; i < 3; i++) n[i] = -n[i];
  int64_t m = 0;
  for (int i = 0; i < 3; i++) {
    int64_t a = n[i] < 0 ? -n[i] : n[i];
    if (a > m) m = a;
  }
  for (int i = 0; i < 3; i++) {
    int64_t a = n[i] < 0 ? -n[i] : n[i];
    if (a != 0 && a != m) return -1;
    un[i] = (int32_t)(n[i] / m);
  }
  for (int d = 0; d < 9; d++) {
    if (un[0] == or_dirs[d][0] && un[1] == or_dirs[d][1] && un[2] == or_dirs[d][2]) {
      *off = un[0] * v[idx[0]][0] + un[1] * v[idx[0]][1] + un[2] * v[idx[0]][2];
      return 2 * d;
    }
    if (un[0] == -or_dirs[d][0] && un[1] == -or_dirs[d][1] && un[2] == -or_dirs[d][2]) {
      *off = un[0] * v[idx[0]][0] + un[1] * v[idx[0]][1] + un[2] * v[idx[0]][2];
      return 2 * d + 1;
    }
  }
  return -1;
}

typedef struct { uint64_t k[3]; int64_t tet; int32_t face; int32_t used; } face_ent;

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int on_boundary(const int32_t* a, const int32_t* b, const int32_t* c) {
  for (int i = 0; i < 3; i++)
    if (a[i] == b[i] && b[i] == c[i] && (a[i] == 0 || a[i] == OR_LAT_S)) return 1;
  return 0;
}

static int build_neighbours(ogrid* g) {
  uint64_t cap = 1;
  while (cap < (uint64_t)g->n * 8) cap <<= 1;
  face_ent* ft = (face_ent*)calloc((size_t)cap, sizeof(face_ent));
  if (!ft) return -2;
  for (int64_t t = 0; t < g->n * 4; t++) g->nbr[t] = OR_BOUNDARY;
  int rc = 0;
  for (int64_t t = 0; t < g->n && !rc; t++) {
    const int32_t(*v)[3] = (const int32_t(*)[3])(g->verts + 12 * t);
    for (int f = 0; f < 4; f++) {
      uint64_t k[3];
      int q = 0;
      for (int j = 0; j < 4; j++)
        if (j != f) k[q++] = vkey(v[j]);
      qsort(k, 3, sizeof(uint64_t), cmp_u64);
      uint64_t h = or_mix64(k[0] ^ or_mix64(k[1] ^ or_mix64(k[2]))) & (cap - 1);
      for (;;) {
        face_ent* e = &ft[h];
        if (!e->used) {
          e->used = 1;
          memcpy(e->k, k, sizeof(k));
          e->tet = t;
          e->face = f;
          break;
        }
        if (e->k[0] == k[0] && e->k[1] == k[1] && e->k[2] == k[2]) {
          if (e->used == 2) { rc = -7; break; } /* third tet on one face */
          e->used = 2;
          g->nbr[4 * t + f] = ((uint32_t)e->tet << 2) | (uint32_t)e->face;
          g->nbr[4 * e->tet + e->face] = ((uint32_t)t << 2) | (uint32_t)f;
          break;
        }
        h = (h + 1) & (cap - 1);
      }
    }
  }
  /* every unmatched face must lie on the cube boundary */
  for (int64_t t = 0; t < g->n && !rc; t++) {
    const int32_t(*v)[3] = (const int32_t(*)[3])(g->verts + 12 * t);
    for (int f = 0; f < 4; f++) {
      if (g->nbr[4 * t + f] != OR_BOUNDARY) continue;
      int idx[3], q = 0;
      for (int j = 0; j < 4; j++)
        if (j != f) idx[q++] = j;
      if (!on_boundary(v[idx[0]], v[idx[1]], v[idx[2]])) { rc = -7; break; }
    }
  }
  free(ft);
  return rc;
}

static int build_id_hash(ogrid* g) {
  uint64_t cap = 1;
  while (cap < (uint64_t)g->n * 2 + 2) cap <<= 1;
  g->hcap = cap;
  g->hkeys = (uint64_t*)calloc((size_t)cap, sizeof(uint64_t));
  g->hvals = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
  if (!g->hkeys || !g->hvals) return -2;
  for (int64_t t = 0; t < g->n; t++) {
    uint64_t h = or_mix64(g->ids[t]) & (cap - 1);
    while (g->hkeys[h]) h = (h + 1) & (cap - 1);
    g->hkeys[h] = g->ids[t];
    g->hvals[h] = t;
  }
  return 0;
}

int64_t or_lookup_id(const ogrid* g, uint64_t id) {
  uint64_t h = or_mix64(id) & (g->hcap - 1);
  while (g->hkeys[h]) {
    if (g->hkeys[h] == id) return g->hvals[h];
    h = (h + 1) & (g->hcap - 1);
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* Build                                                                */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t key; int64_t node; } keyed;

static int cmp_keyed(const void* a, const void* b) {
  uint64_t x = ((const keyed*)a)->key, y = ((const keyed*)b)->key;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int check_inputs(const float* density, int32_t n, const ocam* cam, const obuild_opts* o, int* L) {
  if (!density || !cam || !o || n < 1 || n > (1 << 12) || (n & (n - 1))) return -1;
  if (cam->width < 1 || cam->height < 1 || !(cam->fov_y_deg > 0.0f && cam->fov_y_deg < 180.0f)) return -1;
  if (o->want_mode < 0 || o->want_mode > 2 || o->max_tets < 6) return -1;
  if (o->max_depth < 0 || o->max_depth > 56 || o->uniform_depth < 0 || o->uniform_depth > 56) return -1;
  int l = 0;
  while ((1 << l) < n) l++;
  *L = l;
  int64_t nv = (int64_t)n * n * n;
  for (int64_t i = 0; i < nv; i++)
    if (!(density[i] >= 0.0f) || isinf(density[i])) return -5;
  return 0;
}

int oracle_leb_build(const float* density, int32_t n, const ocam* cam, const obuild_opts* opts, ogrid** out) {
  if (!out) return -1;
  *out = NULL;
  int L = 0;
  int rc = check_inputs(density, n, cam, opts, &L);
  if (rc) return rc;
  bctx c;
  memset(&c, 0, sizeof(c));
  c.dens = density;
  c.n = n;
  c.L = L;
  c.cam = *cam;
  c.o = *opts;
  rc = build_pyramid(&c);
  if (rc) { free_pyramid(&c); return rc; }
  camera_frame(&c);
  for (int r = 0; r < 6; r++) {
    int64_t t = new_node(&c);
    onode* p = &c.nd[t];
    memset(p->v, 0, sizeof(p->v));
    p->v[1][kuhn_perm[r][0]] = OR_LAT_S;
    p->v[2][kuhn_perm[r][0]] = OR_LAT_S;
    p->v[2][kuhn_perm[r][1]] = OR_LAT_S;
    p->v[3][0] = p->v[3][1] = p->v[3][2] = OR_LAT_S;
    p->id = 8 + (uint64_t)r;
    p->depth = 0;
    p->alive = 1;
    edge_attach(&c, t);
  }
  c.nleaves = 6;
  int64_t* wl = NULL;
  int64_t wcap = 0;
  uint64_t shuf = opts->shuffle_seed;
  while (!c.err) {
    int64_t nw = 0;
    int64_t upto = c.nn;
    for (int64_t i = 0; i < upto; i++) {
      onode* t = &c.nd[i];
      if (!t->alive || t->checked) continue;
      t->checked = 1;
      if (!want(&c, (const int32_t(*)[3])t->v, t->depth, t->id)) continue;
      if (nw == wcap) {
        wcap = wcap ? wcap * 2 : 1024;
        int64_t* p = (int64_t*)realloc(wl, (size_t)wcap * sizeof(int64_t));
        if (!p) { c.err = -2; break; }
        wl = p;
      }
      wl[nw++] = i;
    }
    if (c.err || nw == 0) break;
    if (shuf) { /* Fisher-Yates with a splitmix stream */
      for (int64_t i = nw - 1; i > 0; i--) {
        shuf = or_mix64(shuf + 0x9E3779B97F4A7C15ull);
        int64_t j = (int64_t)(shuf % (uint64_t)(i + 1));
        int64_t tmp = wl[i];
        wl[i] = wl[j];
        wl[j] = tmp;
      }
    }
    for (int64_t i = 0; i < nw && !c.err; i++) {
      refine(&c, wl[i], 0);
      if (c.nleaves > opts->max_tets) c.err = -3;
    }
  }
  free(wl);
  if (c.err) {
    free(c.nd);
    free(c.et);
    free_pyramid(&c);
    return c.err;
  }
  /* collect leaves in depth-first order */
  ogrid* g = (ogrid*)calloc(1, sizeof(ogrid));
  keyed* ks = (keyed*)malloc((size_t)c.nleaves * sizeof(keyed));
  if (!g || !ks) { free(g); free(ks); free(c.nd); free(c.et); free_pyramid(&c); return -2; }
  int64_t q = 0;
  for (int64_t i = 0; i < c.nn; i++)
    if (c.nd[i].alive) {
      ks[q].key = dfs_key(c.nd[i].id);
      ks[q].node = i;
      q++;
    }
  qsort(ks, (size_t)q, sizeof(keyed), cmp_keyed);
  g->n = q;
  g->ids = (uint64_t*)malloc((size_t)q * sizeof(uint64_t));
  g->verts = (int32_t*)malloc((size_t)q * 12 * sizeof(int32_t));
  g->nbr = (uint32_t*)malloc((size_t)q * 4 * sizeof(uint32_t));
  g->sigma = (float*)malloc((size_t)q * sizeof(float));
  g->majorant = (float*)malloc((size_t)q * sizeof(float));
  g->codes = (uint8_t*)malloc((size_t)q * 4);
  g->offsets = (int32_t*)malloc((size_t)q * 4 * sizeof(int32_t));
  rc = (g->ids && g->verts && g->nbr && g->sigma && g->majorant && g->codes && g->offsets) ? 0 : -2;
  for (int64_t t = 0; t < q && !rc; t++) {
    const onode* p = &c.nd[ks[t].node];
    g->ids[t] = p->id;
    if (p->depth > g->max_depth) g->max_depth = p->depth;
    memcpy(g->verts + 12 * t, p->v, sizeof(p->v));
    int32_t lo[3], hi[3];
    float mn, mx;
    double s, cnt;
    tet_box((const int32_t(*)[3])p->v, lo, hi);
    box_stats(&c, lo, hi, &mn, &mx, &s, &cnt);
    double mean = s / cnt;
    g->sigma[t] = (float)((double)opts->density_scale * mean);
    g->majorant[t] = opts->majorant_mode == 1 ? (float)((double)opts->density_scale * (double)mx) : g->sigma[t];
    for (int f = 0; f < 4; f++) {
      int32_t un[3], off = 0;
      int code = face_code((const int32_t(*)[3])p->v, f, un, &off);
      if (code < 0) { rc = -7; break; }
      g->codes[4 * t + f] = (uint8_t)code;
      g->offsets[4 * t + f] = off;
    }
  }
  free(ks);
  free(c.nd);
  free(c.et);
  free_pyramid(&c);
  if (!rc) rc = build_neighbours(g);
  if (!rc) rc = build_id_hash(g);
  if (rc) { oracle_grid_free(g); return rc; }
  *out = g;
  return 0;
}

int64_t oracle_grid_num_tets(const ogrid* g) { return g ? g->n : -1; }
int32_t oracle_grid_max_depth(const ogrid* g) { return g ? g->max_depth : -1; }

/* Item 8: per-tet means of up to three channel grids (temperature >= 0,
 * albedo in [0, 1], g in (-1, 1); NULL = absent), each n^3 FP32, x
 * fastest, covering the unit cube.  Replaces the grid's channels. */
int oracle_grid_set_channels(ogrid* g, const float* temperature, const float* albedo, const float* gch, int32_t n) {
  if (!g || n < 1 || n > (1 << 12) || (n & (n - 1))) return -1;
  const float* src[3] = {temperature, albedo, gch};
  int L = 0;
  while ((1 << L) < n) L++;
  int64_t nv = (int64_t)n * n * n;
  for (int k = 0; k < 3; k++) {
    if (!src[k]) continue;
    for (int64_t i = 0; i < nv; i++) {
      float x = src[k][i];
      int ok = k == 0 ? (x >= 0.0f && !isinf(x)) : (k == 1 ? (x >= 0.0f && x <= 1.0f) : (x > -1.0f && x < 1.0f));
      if (!ok) return -5;
    }
  }
  for (int k = 0; k < 3; k++) {
    free(g->ch[k]);
    g->ch[k] = NULL;
    if (!src[k]) continue;
    bctx c;
    memset(&c, 0, sizeof(c));
    c.dens = src[k];
    c.n = n;
    c.L = L;
    float* out = (float*)malloc((size_t)g->n * sizeof(float));
    int rc = out ? build_pyramid(&c) : -2;
    if (rc) {
      free(out);
      free_pyramid(&c);
      return -2;
    }
    for (int64_t t = 0; t < g->n; t++) {
      int32_t lo[3], hi[3];
      tet_box((const int32_t(*)[3])(g->verts + 12 * t), lo, hi);
      float mn, mx;
      double sum, cnt;
      box_stats(&c, lo, hi, &mn, &mx, &sum, &cnt);
      out[t] = (float)(sum / cnt);
    }
    free_pyramid(&c);
    g->ch[k] = out;
  }
  return 0;
}

int oracle_grid_export_channels(const ogrid* g, float* temperature, float* albedo, float* gch) {
  if (!g) return -1;
  float* dst[3] = {temperature, albedo, gch};
  for (int k = 0; k < 3; k++) {
    if (!dst[k]) continue;
    if (!g->ch[k]) return -1;
    memcpy(dst[k], g->ch[k], (size_t)g->n * sizeof(float));
  }
  return 0;
}

/* Item 9, model 1: the trilinear sample of the volume at lattice point v
 * (FP64; unscaled). */
static double trilinear_at(const float* dens, int32_t n, const int32_t v[3]) {
  int64_t i0[3], i1[3];
  double f[3];
  for (int a = 0; a < 3; a++) {
    double u = (double)v[a] * (double)n / (double)OR_LAT_S - 0.5; /* voxel-centre coordinates */
    double fl = floor(u);
    f[a] = u - fl;
    int64_t lo = (int64_t)fl, hi = lo + 1;
    i0[a] = lo < 0 ? 0 : (lo > n - 1 ? n - 1 : lo);
    i1[a] = hi < 0 ? 0 : (hi > n - 1 ? n - 1 : hi);
  }
  double cz[2];
  for (int c = 0; c < 2; c++) {
    int64_t z = c ? i1[2] : i0[2];
    double cy[2];
    for (int b = 0; b < 2; b++) {
      int64_t y = b ? i1[1] : i0[1];
      double d0 = (double)dens[i0[0] + (int64_t)n * (y + (int64_t)n * z)];
      double d1 = (double)dens[i1[0] + (int64_t)n * (y + (int64_t)n * z)];
      cy[b] = (1.0 - f[0]) * d0 + f[0] * d1;
    }
    cz[c] = (1.0 - f[1]) * cy[0] + f[1] * cy[1];
  }
  return (1.0 - f[2]) * cz[0] + f[2] * cz[1];
}

/* Item 9, model 1: the affine function through the four vertex values rho
 * (world units): gradient by Cramer's rule on the edge vectors e_k = v_k -
 * v_0 (lattice integers; cross products and the determinant exact in int64),
 * g = (dr1 (e2 x e3) + dr2 (e3 x e1) + dr3 (e1 x e2)) / det * 2^20 with
 * dr_k = rho_k - rho_0, and c0 = rho_0 - g . v_0 (FP64, rounded to FP32). */
static void linear_coefficients(const int32_t v[4][3], const double rho[4], float out[4]) {
  int64_t e[3][3];
  for (int k = 0; k < 3; k++)
    for (int a = 0; a < 3; a++) e[k][a] = (int64_t)v[k + 1][a] - (int64_t)v[0][a];
  int64_t c[3][3]; /* c[k] = e[k+1] x e[k+2] */
  for (int k = 0; k < 3; k++) {
    const int64_t* p = e[(k + 1) % 3];
    const int64_t* q = e[(k + 2) % 3];
    c[k][0] = p[1] * q[2] - p[2] * q[1];
    c[k][1] = p[2] * q[0] - p[0] * q[2];
    c[k][2] = p[0] * q[1] - p[1] * q[0];
  }
  int64_t det = e[0][0] * c[0][0] + e[0][1] * c[0][1] + e[0][2] * c[0][2];
  double dr[3] = {rho[1] - rho[0], rho[2] - rho[0], rho[3] - rho[0]};
  double g[3];
  for (int a = 0; a < 3; a++)
    g[a] = ((dr[0] * (double)c[0][a] + dr[1] * (double)c[1][a]) + dr[2] * (double)c[2][a]) / (double)det *
           (double)OR_LAT_S;
  double p0[3] = {(double)v[0][0] / OR_LAT_S, (double)v[0][1] / OR_LAT_S, (double)v[0][2] / OR_LAT_S};
  double c0 = rho[0] - ((g[0] * p0[0] + g[1] * p0[1]) + g[2] * p0[2]);
  out[0] = (float)c0;
  out[1] = (float)g[0];
  out[2] = (float)g[1];
  out[3] = (float)g[2];
}

int oracle_grid_set_density_model(ogrid* g, const float* density, int32_t n, float scale, int32_t model) {
  if (!g || model < 0 || model > 2) return -1;
  if (model != 0) {
    if (!density || n < 1 || n > (1 << 12) || (n & (n - 1)) || !(scale > 0.0f) || isinf(scale)) return -1;
    int64_t nv = (int64_t)n * n * n;
    for (int64_t i = 0; i < nv; i++)
      if (!(density[i] >= 0.0f) || isinf(density[i])) return -5;
  }
  free(g->mmaj);
  free(g->mcoef);
  free(g->mdens);
  g->mmaj = g->mcoef = g->mdens = NULL;
  g->model = 0;
  if (model == 0) return 0;
  int64_t nv = (int64_t)n * n * n;
  float* maj = (float*)malloc((size_t)g->n * sizeof(float));
  float* coef = model == 1 ? (float*)malloc((size_t)g->n * 4 * sizeof(float)) : NULL;
  float* dcopy = model == 2 ? (float*)malloc((size_t)nv * sizeof(float)) : NULL;
  if (!maj || (model == 1 && !coef) || (model == 2 && !dcopy)) {
    free(maj);
    free(coef);
    free(dcopy);
    return -2;
  }
  int64_t vs = (int64_t)OR_LAT_S / n;
  for (int64_t t = 0; t < g->n; t++) {
    const int32_t(*v)[3] = (const int32_t(*)[3])(g->verts + 12 * t);
    if (model == 1) {
      double rho[4], mx = 0.0;
      for (int j = 0; j < 4; j++) {
        rho[j] = (double)scale * trilinear_at(density, n, v[j]);
        if (j == 0 || rho[j] > mx) mx = rho[j];
      }
      maj[t] = (float)mx;
      linear_coefficients(v, rho, coef + 4 * t);
    } else {
      /* largest voxel over the open bounding box, by direct scan */
      int32_t lo[3], hi[3];
      tet_box(v, lo, hi);
      int64_t r0[3], r1[3];
      for (int a = 0; a < 3; a++) {
        r0[a] = lo[a] / vs;
        r1[a] = (hi[a] + vs - 1) / vs;
      }
      float mx = 0.0f;
      for (int64_t k = r0[2]; k < r1[2]; k++)
        for (int64_t j = r0[1]; j < r1[1]; j++)
          for (int64_t i = r0[0]; i < r1[0]; i++) {
            float x = density[i + (int64_t)n * (j + (int64_t)n * k)];
            if (x > mx) mx = x;
          }
      maj[t] = (float)((double)scale * (double)mx);
    }
  }
  if (dcopy) memcpy(dcopy, density, (size_t)nv * sizeof(float));
  g->mmaj = maj;
  g->mcoef = coef;
  g->mdens = dcopy;
  g->mn = n;
  g->mscale = scale;
  g->model = model;
  return 0;
}

int oracle_grid_export_density_model(const ogrid* g, float* majorant, float* coef) {
  if (!g) return -1;
  if (g->model == 0) return -1;
  if (majorant) memcpy(majorant, g->mmaj, (size_t)g->n * sizeof(float));
  if (coef) {
    if (g->model != 1) return -1;
    memcpy(coef, g->mcoef, (size_t)g->n * 4 * sizeof(float));
  }
  return 0;
}

int oracle_grid_export(const ogrid* g, uint64_t* ids, int32_t* verts, uint32_t* nbr, float* sigma,
                       float* majorant, uint8_t* codes, int32_t* offsets) {
  if (!g) return -1;
  size_t n = (size_t)g->n;
  if (ids) memcpy(ids, g->ids, n * sizeof(uint64_t));
  if (verts) memcpy(verts, g->verts, n * 12 * sizeof(int32_t));
  if (nbr) memcpy(nbr, g->nbr, n * 4 * sizeof(uint32_t));
  if (sigma) memcpy(sigma, g->sigma, n * sizeof(float));
  if (majorant) memcpy(majorant, g->majorant, n * sizeof(float));
  if (codes) memcpy(codes, g->codes, n * 4);
  if (offsets) memcpy(offsets, g->offsets, n * 4 * sizeof(int32_t));
  return 0;
}

void oracle_grid_free(ogrid* g) {
  if (!g) return;
  free(g->ids);
  free(g->verts);
  free(g->nbr);
  free(g->sigma);
  free(g->majorant);
  free(g->codes);
  free(g->offsets);
  free(g->hkeys);
  free(g->hvals);
  for (int k = 0; k < 3; k++) free(g->ch[k]);
  free(g->mmaj);
  free(g->mcoef);
  free(g->mdens);
  free(g);
}

int oracle_box_stats(const float* density, int32_t n, const int32_t lo[3], const int32_t hi[3], float* mn,
                     float* mx, double* sum, double* count) {
  ocam cam = {{0, 0, -1}, {0, 0, 0}, {0, 1, 0}, 45.0f, 1, 1};
  obuild_opts o;
  memset(&o, 0, sizeof(o));
  o.max_tets = 6;
  int L = 0;
  int rc = check_inputs(density, n, &cam, &o, &L);
  if (rc) return rc;
  for (int a = 0; a < 3; a++)
    if (lo[a] < 0 || hi[a] > OR_LAT_S || lo[a] >= hi[a]) return -1;
  bctx c;
  memset(&c, 0, sizeof(c));
  c.dens = density;
  c.n = n;
  c.L = L;
  rc = build_pyramid(&c);
  if (!rc) box_stats(&c, lo, hi, mn, mx, sum, count);
  free_pyramid(&c);
  return rc;
}

int oracle_want(const float* density, int32_t n, const ocam* cam, const obuild_opts* opts, int64_t count,
                const int32_t* verts, const int32_t* depth, const uint64_t* ids, uint8_t* out) {
  int L = 0;
  int rc = check_inputs(density, n, cam, opts, &L);
  if (rc) return rc;
  if (count < 0 || (count && (!verts || !depth || !ids || !out))) return -1;
  bctx c;
  memset(&c, 0, sizeof(c));
  c.dens = density;
  c.n = n;
  c.L = L;
  c.cam = *cam;
  c.o = *opts;
  rc = build_pyramid(&c);
  if (!rc) {
    camera_frame(&c);
    for (int64_t i = 0; i < count; i++)
      out[i] = (uint8_t)want(&c, (const int32_t(*)[3])(verts + 12 * i), depth[i], ids[i]);
  }
  free_pyramid(&c);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Point location                                                       */
/* ------------------------------------------------------------------ */
/* Root: the Kuhn tet whose axis order sorts the point's coordinates in
 * descending order (first such root on ties).  Descent: the first child
 * keeps x0; p goes to it iff n.(p - z) >= 0, n the unit normal of the
 * bisection plane (through z and the two other vertices) oriented toward
 * x0, evaluated in FP64 on the lattice-scaled point. */
int64_t or_locate_point(const ogrid* g, const float p[3]) {
  int r = -1;
  for (int q = 0; q < 6 && r < 0; q++) {
    const int* pm = kuhn_perm[q];
    if (p[pm[0]] >= p[pm[1]] && p[pm[1]] >= p[pm[2]]) r = q;
  }
  if (r < 0) return -1;
  int32_t v[4][3];
  memset(v, 0, sizeof(v));
  v[1][kuhn_perm[r][0]] = OR_LAT_S;
  v[2][kuhn_perm[r][0]] = OR_LAT_S;
  v[2][kuhn_perm[r][1]] = OR_LAT_S;
  v[3][0] = v[3][1] = v[3][2] = OR_LAT_S;
  uint64_t id = 8 + (uint64_t)r;
  int depth = 0;
  double P[3];
  for (int i = 0; i < 3; i++) P[i] = (double)p[i] * (double)OR_LAT_S;
  for (;;) {
    int64_t t = or_lookup_id(g, id);
    if (t >= 0) return t;
    if (depth >= 60) return -1;
    int k = tag_of(depth);
    int32_t z[3];
    for (int i = 0; i < 3; i++) z[i] = (v[0][i] + v[k][i]) / 2;
    int j1 = -1, j2 = -1;
    for (int j = 1; j < 4; j++)
      if (j != k) { if (j1 < 0) j1 = j; else j2 = j; }
    int64_t a[3], b[3], nn[3];
    for (int i = 0; i < 3; i++) {
      a[i] = (int64_t)v[j1][i] - z[i];
      b[i] = (int64_t)v[j2][i] - z[i];
    }
    nn[0] = a[1] * b[2] - a[2] * b[1];
    nn[1] = a[2] * b[0] - a[0] * b[2];
    nn[2] = a[0] * b[1] - a[1] * b[0];
    int64_t s0 = 0;
    for (int i = 0; i < 3; i++) s0 += nn[i] * ((int64_t)v[0][i] - z[i]);
    double side = 0.0;
    for (int i = 0; i < 3; i++) {
      int sg = nn[i] > 0 ? 1 : (nn[i] < 0 ? -1 : 0);
      if (s0 < 0) sg = -sg;
      if (sg) side = side + (double)sg * (P[i] - (double)z[i]);
    }
    int32_t w[4][3];
    if (side >= 0.0) {
      memcpy(w, v, sizeof(w));
      memcpy(w[k], z, sizeof(z));
      id = 2 * id;
    } else {
      for (int j = 0; j < k; j++) memcpy(w[j], v[j + 1], sizeof(z));
      memcpy(w[k], z, sizeof(z));
      for (int j = k + 1; j < 4; j++) memcpy(w[j], v[j], sizeof(z));
      id = 2 * id + 1;
    }
    memcpy(v, w, sizeof(w));
    depth++;
  }
}

int oracle_locate(const ogrid* g, int64_t count, const float* pts, int64_t* out) {
  if (!g || count < 0 || (count && (!pts || !out))) return -1;
  for (int64_t i = 0; i < count; i++) {
    const float* p = pts + 3 * i;
    int ok = 1;
    for (int a = 0; a < 3; a++)
      if (!(p[a] >= 0.0f && p[a] <= 1.0f)) ok = 0;
    out[i] = ok ? or_locate_point(g, p) : -1;
  }
  return 0;
}
