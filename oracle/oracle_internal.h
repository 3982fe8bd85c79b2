/* oracle_internal.h -- grid object shared by the oracle's own source files.
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include "oracle.h"
#include <stddef.h>

#define OR_LAT_BITS 20
#define OR_LAT_S (1 << OR_LAT_BITS) /* lattice units per world unit */
#define OR_BOUNDARY 0xFFFFFFFFu

struct ogrid {
  int64_t n;              /* number of tets (leaves) */
  int32_t max_depth;
  uint64_t* ids;          /* heap ids, sorted by depth-first key */
  int32_t* verts;         /* 12 per tet, lattice units */
  uint32_t* nbr;          /* 4 per tet: (index << 2) | back face, or OR_BOUNDARY */
  float* sigma;           /* extinction per tet */
  float* majorant;        /* per-tet majorant (>= sigma) */
  uint8_t* codes;         /* 4 per tet: outward face orientation code */
  int32_t* offsets;       /* 4 per tet: lattice plane offset */
  /* optional extra channels per tet (NULL = absent): temperature, albedo,
   * phase parameter g -- each the mean over the tet's voxel box */
  float* ch[3];
  /* density model inside each tet (leb.c item 9): 0 constant (sigma above),
   * 1 linear, 2 voxel lookup; per-tet majorant; model 1: 4 coefficients per
   * tet (c0, gx, gy, gz); model 2: a copy of the n^3 volume and its scale */
  int32_t model;
  float* mmaj;
  float* mcoef;
  float* mdens;
  int32_t mn;
  float mscale;
  /* id -> canonical index (open addressing) */
  uint64_t* hkeys;
  int64_t* hvals;
  uint64_t hcap;
};

/* The 9 plane directions a face of these grids can have; code = 2*N + s
 * where the outward normal is +dir[N] (s = 0) or -dir[N] (s = 1). */
extern const int32_t or_dirs[9][3];

uint64_t or_mix64(uint64_t x);
int64_t  or_lookup_id(const ogrid* g, uint64_t id);
int64_t  or_locate_point(const ogrid* g, const float p[3]);

#endif
