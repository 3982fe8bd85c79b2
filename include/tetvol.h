/*
 * tetvol.h -- C ABI of libtetvol.so: adaptive tetrahedral grids for
 * volumetric path tracing on MI355X (gfx950).
 *
 * Method: Benyoub & Dupuy, "Adaptive Tetrahedral Grids for Volumetric
 * Path-Tracing", SIGGRAPH Talks 2025.  The library builds an adaptive,
 * conforming tetrahedral grid from a dense density volume by longest-edge
 * bisection (paper, "Grid Construction") and path-traces it by walking tets
 * through their face neighbours (paper, "Volumetric Path Tracing",
 * Algorithm 1, and "Path Tracing within Tetrahedral Grids").
 *
 * General conventions (every entry point):
 *   - Return value: TET_OK (0) or a negative tet_status.  On error nothing is
 *     written to the outputs and *out handles stay NULL; tet_last_error()
 *     returns a message for the calling thread's last failure.
 *   - The caller owns every input and output buffer; the library owns
 *     handles (free them with the matching *_free).  No buffer is retained
 *     after a call returns.
 *   - `on_device` != 0 marks a pointer as device memory of the current HIP
 *     device (e.g. a torch CUDA tensor's data_ptr()); 0 marks host memory.
 *   - `hip_stream` is a hipStream_t or NULL (the null stream).  Calls are
 *     synchronous with respect to the host: outputs are complete on return.
 *   - Handles are bound to the device that was current when they were made.
 *   - Calls on one handle must not overlap; distinct handles may be used
 *     from different threads.
 */
#ifndef TETVOL_H
#define TETVOL_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TET_OK = 0,
  TET_ERR_INVALID_ARG = -1,   /* NULL pointer, bad size or option */
  TET_ERR_OUT_OF_MEMORY = -2, /* device or host allocation failed */
  TET_ERR_CAPACITY = -3,      /* grid would exceed max_tets */
  TET_ERR_DEVICE = -4,        /* a HIP call failed */
  TET_ERR_NUMERIC = -5,       /* NaN, infinite or negative density */
  TET_ERR_UNSUPPORTED = -6,   /* option not supported by this build */
  TET_ERR_INTERNAL = -7       /* invariant violated (non-conforming mesh) */
} tet_status;

typedef struct tet_grid tet_grid; /* device-resident grid, library-owned */
typedef struct tet_nrc tet_nrc;   /* radiance-cache state, library-owned */

/* Dense density volume: n^3 FP32 values, voxel (i,j,k) at index
 * i + n (j + n k), covering [i/n,(i+1)/n) x ... of the unit cube (the
 * paper's control cube fitted to the volume).  n is a power of two,
 * 1 <= n <= 4096.  Values must be finite and >= 0.  Extinction =
 * density_scale * density. */
typedef struct {
  const float* data;
  int32_t n;
  int32_t on_device;
  float density_scale;
} tet_density;

/* Pinhole camera.  Row 0 of an image is its top row. */
typedef struct {
  float pos[3], look_at[3], up[3];
  float fov_y_deg; /* vertical field of view, (0, 180) */
  int32_t width, height;
} tet_camera;

/* Homogeneous scattering properties: single-scattering albedo in [0,1]
 * and Henyey-Greenstein asymmetry g in (-1, 1). */
typedef struct { float albedo, g; } tet_medium;

/* One directional light (sun_dir points toward the light, unit length)
 * and a constant environment seen by paths leaving the grid. */
typedef struct {
  float sun_dir[3];
  float sun_irradiance[3];
  float env_radiance[3];
} tet_light;

typedef struct {
  /* 0: the paper's two criteria (density variation and camera);
   * 1: uniform refinement to uniform_depth;
   * 2: test mode, split iff mix64(id ^ rand_seed) mod 2^16 < rand_thresh
   *    and depth < max_depth (mix64 = the splitmix64 finaliser). */
  int32_t want_mode;
  int32_t uniform_depth;
  int32_t max_depth;       /* depth cap of the criteria (<= 56) */
  int32_t majorant_mode;   /* 0: majorant = extinction (tight); 1: scale*max(D) */
  double variation_tau;    /* split iff (max D - min D) > tau * mean D */
  int64_t max_tets;        /* capacity; TET_ERR_CAPACITY beyond it */
  uint64_t rand_seed;
  int32_t rand_thresh;
  int32_t reserved;
} tet_build_opts;

typedef struct {
  int32_t max_bounces;        /* real collisions per path, >= 1 */
  int32_t transmittance;      /* light: 0 analytic, 1 ratio tracking, 2 delta tracking */
  int64_t max_steps_per_path; /* exit evaluations per path (all walks) */
  int32_t sample_offset;      /* render samples [offset, offset + spp) */
  int32_t samples_per_item;   /* samples one lane takes at a time (0 = all of a pixel) */
  int32_t block_size;         /* threads per block: 64, 128, 192 or 256 (0 = default) */
  int32_t blocks_per_cu;      /* persistent blocks per compute unit (0 = default) */
  int32_t waves_per_simd;     /* register budget of the tracing kernel: 4, 5, 6 or 8 waves (0 = default 5) */
  int32_t record_layout;      /* tet records walked: 32 (compact), 48, or 0 = compact when the grid has them */
  int32_t batch_items;        /* work items a wave takes at a time (0 = default 64) */
  int32_t event_wait;         /* lanes of a wave that wait for an event before events run (0 = default 48) */
} tet_render_opts;

typedef struct {
  int64_t tet_steps;       /* exit evaluations: camera, scattered and light walks */
  int64_t null_collisions;
  int64_t real_collisions;
  int64_t escapes;
  int64_t truncated;       /* paths stopped by max_steps_per_path */
  double ms;               /* device time of the whole render call */
  double trace_ms;         /* device time of the persistent tracing kernel(s) alone */
} tet_render_stats;

typedef struct {
  int32_t rounds;   /* refinement rounds until no tet split */
  int32_t max_depth;
  int64_t num_tets;
  double ms;        /* device time of the whole build */
} tet_build_stats;

void tet_build_opts_defaults(tet_build_opts* o);
void tet_render_opts_defaults(tet_render_opts* o);

/* Builds the adaptive, conforming tet grid (paper, "Grid Construction":
 * longest-edge bisection after Maubach from the control cube, propagation
 * of bisections to keep the grid conforming, subdivision by density
 * variation and by camera -- no split outside the frustum or below
 * target_cell_px projected pixels).  Roots: the 6 Kuhn tets of the unit
 * cube (their depth-2 descendants are the paper's 24 half-edge tets).
 * Tets are ordered by depth-first key (heap id << (60 - depth)).
 * Per tet: one extinction value (scale * mean density over the tet's
 * bounding-box voxels), a majorant, 4 face-neighbour links and 4 face
 * orientation codes (18 orientations).  *out receives a new handle. */
int leb_build(const tet_density* density, const tet_camera* camera, float target_cell_px,
              const tet_build_opts* opts /* NULL = defaults */, void* hip_stream, tet_grid** out);

int tet_grid_info(const tet_grid* grid, int64_t* num_tets, int32_t* max_depth, tet_build_stats* stats);

/* Copies grid arrays out (any pointer may be NULL): ids[num_tets] heap ids;
 * nbr4[num_tets*4] = (index << 2) | back_face, or 0xFFFFFFFF on the
 * boundary; sigma / majorant [num_tets]; verts12[num_tets*12] lattice
 * vertices (world * 2^20). */
int tet_grid_export(const tet_grid* grid, uint64_t* ids, uint32_t* nbr4, float* sigma, float* majorant,
                    int32_t* verts12, int32_t on_device, void* hip_stream);

/* Renders spp samples per pixel of the grid with the Monte Carlo volumetric
 * path tracer (paper, Algorithm 1: enter the grid, then sample a free path,
 * march through cells via face neighbours testing at most 3 faces, sample
 * the phase function) with next-event estimation of the sun and the
 * environment on escape.  out_rgb: width*height*3 FP32, pixel (x, y) at
 * 3 (y width + x), holding the average of the spp samples.  Random numbers
 * come from Philox4x32-10 keyed by seed, so a pixel's value does not
 * depend on the image, tile or launch it is rendered in. */
int tet_render(const tet_grid* grid, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
               int32_t spp, uint64_t seed, const tet_render_opts* opts /* NULL = defaults */, float* out_rgb,
               int32_t on_device, void* hip_stream, tet_render_stats* stats /* nullable */);

/* Point location (the grid-entry step of Algorithm 1): canonical index of
 * the tet containing each point (3 FP32 per point, inside [0,1]^3), or -1.
 * pts and out live on the same side (on_device). */
int tet_locate(const tet_grid* grid, const float* pts, int64_t count, int64_t* out, int32_t on_device,
               void* hip_stream);

/* The same integrator on the regular voxel grid (the paper's regular-grid
 * reference renderer), voxels walked by Amanatides-Woo traversal. */
int dda_render(const tet_density* density, const tet_camera* camera, const tet_medium* medium,
               const tet_light* light, int32_t spp, uint64_t seed, const tet_render_opts* opts, float* out_rgb,
               int32_t on_device, void* hip_stream, tet_render_stats* stats);

void tet_grid_free(tet_grid* grid);

/* Frees device memory cached by the library between calls. */
void tet_release_cache(void);

const char* tet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
