/*
 * oracle.h -- plain, slow CPU statement of the adaptive tetrahedral grid
 * method (Benyoub & Dupuy, "Adaptive Tetrahedral Grids for Volumetric
 * Path-Tracing", SIGGRAPH Talks 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load liboracle.so.  It shares no source, header,
 * table or constant generator with the HIP path.
 *
 * Section map (paper):
 *   Grid Construction / Longest Edge Bisection  -> leb.c   (roots, Maubach
 *       bisection, conforming closure, neighbour table, face codes)
 *   Grid Construction / Subdivision Criteria    -> leb.c   (density
 *       statistics, density-variation and camera criteria)
 *   Volumetric Path Tracing / Algorithm 1 and
 *   "Path Tracing within Tetrahedral Grids"     -> transport.c
 *   (not in the paper) MLP radiance cache       -> mlp.c
 *
 * Readings of passages the paper leaves open are stated at each function.
 * All functions return 0 on success and a negative status on error:
 *   -1 invalid argument, -2 out of memory, -3 capacity, -5 numeric
 *   (NaN / negative density), -7 non-conforming mesh detected.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same field layout as the product's camera / medium / light structs (an
 * interface that has to be alike); declared here independently. */
typedef struct { float pos[3], look_at[3], up[3]; float fov_y_deg; int32_t width, height; } ocam;
typedef struct { float albedo, g; } omedium;
typedef struct { float sun_dir[3]; float sun_irradiance[3]; float env_radiance[3]; } olight;

typedef struct ogrid ogrid;

/* want_mode: 0 = paper criteria (density variation and camera),
 *            1 = uniform to depth `uniform_depth`,
 *            2 = test mode: split iff mix64(id ^ rand_seed) mod 2^16 <
 *                rand_thresh and depth < max_depth (random adaptive marks).
 * shuffle_seed != 0 randomises the order in which wanted leaves are refined
 * (the final grid must not depend on it). */
typedef struct {
  int32_t want_mode;
  int32_t uniform_depth;
  int32_t max_depth;
  int32_t majorant_mode;      /* 0 tight (majorant = sigma), 1 = scale * max(D) */
  double  variation_tau;
  float   target_px;
  float   density_scale;
  int64_t max_tets;
  uint64_t rand_seed;
  int32_t rand_thresh;
  uint64_t shuffle_seed;
} obuild_opts;

int  oracle_leb_build(const float* density, int32_t n, const ocam* cam,
                      const obuild_opts* opts, ogrid** out);
int64_t oracle_grid_num_tets(const ogrid* g);
int32_t oracle_grid_max_depth(const ogrid* g);
/* Any output pointer may be NULL.  Arrays are indexed by the canonical tet
 * index (leaves sorted by depth-first key).  verts: 12 int32 per tet (lattice
 * units, S = 2^20).  nbr: 4 uint32 per tet, (index << 2) | back_face, or
 * 0xFFFFFFFF on the boundary.  codes: 4 uint8 per tet (face orientation code
 * 0..17).  offsets: 4 int32 per tet (lattice plane offset n_f . v). */
int  oracle_grid_export(const ogrid* g, uint64_t* ids, int32_t* verts, uint32_t* nbr,
                        float* sigma, float* majorant, uint8_t* codes, int32_t* offsets);
void oracle_grid_free(ogrid* g);

/* Density statistics of a lattice box [lo, hi] (lattice units): min, max,
 * FP64 sum in the pyramid's order, voxel count. */
int  oracle_box_stats(const float* density, int32_t n, const int32_t lo[3], const int32_t hi[3],
                      float* mn, float* mx, double* sum, double* count);
/* Want predicate for arbitrary tets given by vertices (12 int32 each) and
 * depth. */
int  oracle_want(const float* density, int32_t n, const ocam* cam, const obuild_opts* opts,
                 int64_t count, const int32_t* verts, const int32_t* depth, const uint64_t* ids,
                 uint8_t* out);

/* Point location: canonical tet index containing each point (world units,
 * FP32, inside [0,1]^3), or -1. */
int  oracle_locate(const ogrid* g, int64_t count, const float* pts, int64_t* out);

/* One walk of a straight segment (origin o, direction d, start tet) until the
 * boundary or max_out steps: tet sequence, exit faces and exit distances. */
/* Extra channels per tet (leb.c item 8); NULL channel = absent. */
int  oracle_grid_set_channels(ogrid* g, const float* temperature, const float* albedo, const float* gch, int32_t n);
int  oracle_grid_export_channels(const ogrid* g, float* temperature, float* albedo, float* gch);

/* Density model inside the tets (leb.c item 9): model 0 constant per tet,
 * 1 linear between trilinear vertex samples of `density` (n^3, x fastest),
 * 2 the voxel of `density` containing the point; `scale` multiplies the
 * density.  Export: per-tet majorant, and for model 1 the coefficients
 * (c0, gx, gy, gz) of sigma(x) = ((c0 + gx x) + gy y) + gz z. */
int  oracle_grid_set_density_model(ogrid* g, const float* density, int32_t n, float scale, int32_t model);
int  oracle_grid_export_density_model(const ogrid* g, float* majorant, float* coef);

int  oracle_walk(const ogrid* g, const float o[3], const float d[3], int64_t start,
                 int32_t max_out, int64_t* tets, int32_t* faces, float* texit, int32_t* n_out);

typedef struct {
  int32_t max_bounces;
  int32_t transmittance;      /* 0 analytic, 1 ratio tracking, 2 delta tracking */
  int64_t max_steps_per_path;
  int32_t sample_offset;
  int32_t channels;           /* 1: use the grid's extra channels (transport.c) */
  float emission[3];          /* radiance emitted per unit temperature (RGB) */
} orender_opts;

typedef struct { int64_t tet_steps, null_collisions, real_collisions, escapes, truncated; } orender_stats;

/* Renders the listed pixels (pixel index = row * width + col, row 0 = top);
 * pixels == NULL renders the whole image in raster order.  out_rgb holds
 * 3 floats per rendered pixel.  threads <= 1 runs single-threaded. */
int  oracle_tet_render(const ogrid* g, const ocam* cam, const omedium* med, const olight* light,
                       int32_t spp, uint64_t seed, const orender_opts* opts,
                       const int32_t* pixels, int64_t n_pixels, float* out_rgb,
                       orender_stats* stats, int32_t threads);

/* Same integrator on the regular voxel grid (Amanatides-Woo traversal). */
int  oracle_dda_render(const float* density, int32_t n, float density_scale, const ocam* cam,
                       const omedium* med, const olight* light, int32_t spp, uint64_t seed,
                       const orender_opts* opts, const int32_t* pixels, int64_t n_pixels,
                       float* out_rgb, orender_stats* stats, int32_t threads);

/* Building blocks exposed for pinning. */
void  oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float oracle_uniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce,
                     uint32_t stream, uint32_t draw);
float oracle_hg_sample_mu(float g, float u);
float oracle_neglog1m(float u);
float oracle_expneg(float x);
void  oracle_sincos2pi(float u, float* c, float* s);
float oracle_hg_eval(float g, float mu);
void  oracle_hg_direction(const float d[3], float g, float u1, float u2, float out[3]);
void  oracle_camera_ray(const ocam* cam, int32_t px, int32_t py, float u0, float u1,
                        float o[3], float d[3]);

/* MLP radiance cache (not in the paper): 76 -> 64 x4 (ReLU) -> 3 (linear).
 * params layout (17,603 values): for each layer l: W_l row-major
 * [out][in] then b_l[out].  bf16 != 0 rounds every matrix-product operand
 * to bfloat16 (see mlp.c). */
float oracle_bf16_round(float x);
int  oracle_nrc_encode(int64_t count, const float* pos, const float* dir, const float* sigma, float sigma_ref,
                       float* feats /* count x 76 */);
int  oracle_mlp_forward(const double* params, int64_t count, const double* x /* count x 76 */,
                        double* y /* count x 3 */, int32_t bf16);
int  oracle_mlp_backward(const double* params, int64_t count, const double* x,
                         const double* dy /* count x 3 */, double* y, double* grads, int32_t bf16);
int  oracle_nrc_loss_grad(int64_t count, const double* y, const double* target, double* loss,
                          double* dy);
int  oracle_adam_step(int64_t n, double* params, const double* grads, double* m, double* v,
                      int64_t step, double lr, double beta1, double beta2, double eps);
int  oracle_ema_step(int64_t n, double* ema, const double* params, double beta, int64_t step, double* out);
void oracle_nrc_eval_point(const double* params, int32_t bf16, float sigma_ref, const float p[3],
                           const float d[3], float sigma, float out[3]);
/* Truncated render with the cache, training pixel choice and training
 * records (transport.c). */
int  oracle_nrc_render(const ogrid* g, const ocam* cam, const omedium* med, const olight* light, int32_t spp,
                       uint64_t seed, const orender_opts* opts, const double* params, int32_t bf16,
                       int32_t truncate_bounce, float sigma_ref, const int32_t* pixels, int64_t n_pixels,
                       float* out_rgb, orender_stats* stats, int32_t threads);
int32_t oracle_train_pixel(uint64_t frame_seed, uint32_t j, int64_t npix);
int  oracle_nrc_collect(const ogrid* g, const ocam* cam, const omedium* med, const olight* light,
                        uint64_t frame_seed, const orender_opts* opts, int32_t n_paths, int32_t max_vertices,
                        float* pos, float* dir, float* sigma, float* target, int32_t* tag, int64_t* count,
                        int32_t* path_pixel, float* path_L, int32_t threads);

#ifdef __cplusplus
}
#endif
#endif
