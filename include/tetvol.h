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
  TET_ERR_UNSUPPORTED = -6,   /* option or combination not supported */
  TET_ERR_INTERNAL = -7       /* invariant violated (non-conforming mesh) */
} tet_status;

typedef struct tet_grid tet_grid; /* device-resident grid, library-owned */
typedef struct tet_nrc tet_nrc;   /* radiance cache (network and optimiser state), library-owned */

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
  int32_t host_rounds;     /* 1: every refinement round is driven from the host; 0 (default): while the
                              grid is small, rounds run inside one cooperative launch.  The grid is the
                              same; profilers that fail on cooperative launches want 1. */
} tet_build_opts;

typedef struct {
  int32_t max_bounces;        /* real collisions per path, >= 1 */
  int32_t transmittance;      /* light: 0 analytic, 1 ratio tracking, 2 delta tracking */
  int64_t max_steps_per_path; /* exit evaluations per path (all walks); default 2^31 - 1.  At that value
                                 (and above), on tet grids without a density model, with analytic light
                                 transmittance, the light rays of a render's passes are queued, sorted by
                                 where they start (column of the grid along the light, then depth) and
                                 walked together after each pass (a light walk then runs on its own,
                                 bounded by the tet count; the estimate is the same unless a path takes
                                 more than 2^31 - 1 steps); their terms reach the pixels apart from the
                                 rest of their samples (FP32 sums in another order).  Grids with extra
                                 channels and the radiance cache's image paths queue theirs too; its
                                 training paths, batches and tet_render_noalloc walk their own */
  int32_t sample_offset;      /* render samples [offset, offset + spp) */
  int32_t samples_per_item;   /* samples one lane takes at a time (0 = all of a pixel) */
  int32_t block_size;         /* threads per block: 64, 128, 192 or 256 (0 = default) */
  int32_t blocks_per_cu;      /* persistent blocks per compute unit (0 = default) */
  int32_t waves_per_simd;     /* register budget of the tracing kernel: 4, 5, 6 or 8 waves (0 = default 5) */
  int32_t record_layout;      /* tet records walked: 32 (compact), 48, or 0 = compact when the grid has them */
  int32_t batch_items;        /* work items a wave takes at a time (0 = default 64; batches always take 64) */
  int32_t event_wait;         /* lanes of a wave that wait for an event before events run (0 = default: 32;
                                 48 when collecting training paths) */
  const tet_nrc* nrc;         /* radiance cache: NULL = plain estimator; else paths stop at the cache's
                                 truncate_bounce-th real vertex and add throughput x cache (tet grids only) */
  int32_t nrc_train;          /* with a cache: the same launch also traces the cache's training paths of
                                 this frame (frame seed = seed XOR 0x6A09E667F3BCC909), then the cache takes
                                 its Adam steps; the image uses the weights from before the call.  The
                                 cache is modified: no other call may use it meanwhile. */
  int32_t channels;           /* 1: use the grid's extra channels (tet_grid_set_channels): a real collision
                                 in tet c adds beta (1 - a_c) T_c emission, then takes the tet's albedo a_c
                                 and phase parameter g_c in place of the medium's (absent channels: the
                                 medium's values, no emission).  Tet grids only; with a radiance cache the
                                 cache at vertex k stands for the vertex's emission too; in batches every
                                 grid must carry channels. */
  float emission[3];          /* radiance emitted per unit temperature (RGB, >= 0), with channels */
} tet_render_opts;

typedef struct {
  int64_t tet_steps;       /* exit evaluations: camera, scattered and light walks */
  int64_t null_collisions;
  int64_t real_collisions;
  int64_t escapes;
  int64_t truncated;       /* paths stopped by max_steps_per_path */
  double ms;               /* device time of the whole render call */
  double trace_ms;         /* device time of the persistent tracing kernel(s) alone */
  double cache_ms;         /* device time of the radiance-cache queries (0 without a cache) */
  int64_t cache_queries;   /* paths that stopped at the cache */
  int64_t cache_records;   /* training records of the frame (nrc_train) */
  double cache_loss;       /* their mean batch loss before the Adam steps (nrc_train) */
  int64_t light_rays_queued; /* light rays walked from the queue (the others: by their own lanes) */
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

/* The same build from a sparse volume (the paper builds from OpenVDB data,
 * "Subdivision Criteria"): the n^3 volume is zero outside num_bricks
 * leaf bricks of 8^3 voxels.  brick_coords: 3 int32 per brick, its position
 * in brick units (voxel / 8) along x, y, z, each in [0, n / 8);
 * brick_values: 512 FP32 per brick, x fastest inside the brick; both on the
 * device or both on the host (on_device).  n is a power of two, 8 <= n <=
 * 4096.  The grid is identical, bit for bit, to leb_build's on the dense
 * volume the bricks describe; the build never holds that dense volume (the
 * pyramid's levels 1 and 2 are kept per brick, levels >= 3 dense).  Errors
 * as leb_build, plus TET_ERR_INVALID_ARG for a brick out of range or listed
 * twice.  The caller's buffers are only read. */
typedef struct {
  const int32_t* brick_coords;
  const float* brick_values;
  int64_t num_bricks;
  int32_t n;
  int32_t on_device;
  float density_scale;
} tet_sparse_density;

int leb_build_sparse(const tet_sparse_density* density, const tet_camera* camera, float target_cell_px,
                     const tet_build_opts* opts, void* hip_stream, tet_grid** out);

/* Rebuilds `grid` in place for a new camera (or density, target or
 * options), starting from the grid's current tree instead of the 6 roots:
 * the real-time use of the paper ("Results": pre-visualisation at
 * interactive rates and animated sequences, where the grid follows the
 * camera, which the camera criterion of "Subdivision Criteria" makes it
 * depend on).  The result is identical, bit for bit, to leb_build (resp.
 * leb_build_sparse) with the same arguments.  Every node of the current
 * tree that the new criteria want, as they want all its ancestors, is
 * split by that build too, so its rounds are continued from those nodes:
 * tets the new criteria no longer want merge back into their first
 * unwanted ancestor, tets they want split further, and the rounds restore
 * conformity.  Arguments and errors as leb_build; on error the grid is
 * unchanged.  Extra channels and density models set on the grid are
 * dropped (they are per tet: set them again).  The grid must live on the
 * current device. */
int leb_update(tet_grid* grid, const tet_density* density, const tet_camera* camera, float target_cell_px,
               const tet_build_opts* opts, void* hip_stream);
int leb_update_sparse(tet_grid* grid, const tet_sparse_density* density, const tet_camera* camera,
                      float target_cell_px, const tet_build_opts* opts, void* hip_stream);

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

/* tet_render for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same render (same kernels, same image up to FP32 summation order),
 * with its scratch -- per-pass entry records and counters -- in a fixed
 * device array of 64 MiB + 256 bytes that the library holds on each device
 * it runs on until the process ends, instead of memory it allocates; the
 * call makes
 * no hipMalloc or hipFree and launches on the stream without waiting (the
 * image is complete once the stream is).  Limits: a tet grid built on the
 * current device, no radiance cache (opts->nrc NULL), out_rgb on the
 * device; one sample of every pixel must fit the array (2^21 entry
 * records: images of up to 2^21 pixels once rounded up to 8 x 8 tiles, e.g.
 * 2048 x 1024), else TET_ERR_CAPACITY; a frame takes ceil(spp / floor(2^21
 * / tiled pixels)) passes.  Every call on a device shares its array: calls that
 * overlap on one device race (serialise them, e.g. on one stream). */
int tet_render_noalloc(const tet_grid* grid, const tet_camera* camera, const tet_medium* medium,
                       const tet_light* light, int32_t spp, uint64_t seed, const tet_render_opts* opts,
                       float* out_rgb, void* hip_stream);

/* Renders n scenes (each its own grid, camera, medium, light, spp and
 * seed) with one persistent launch of the same path tracer: the scenes'
 * samples are work items of one queue, so small images fill the GPU
 * together instead of one after another.  out_rgb[i]: device pointer,
 * width_i*height_i*3 FP32, as tet_render would write it.  Per-scene
 * images equal tet_render's up to FP32 summation order.  opts (nullable):
 * max_bounces, transmittance, max_steps_per_path, sample_offset,
 * block_size, blocks_per_cu, record_layout, event_wait, channels and
 * emission apply to all scenes (with channels, every grid must carry
 * some); a grid's density model renders as in tet_render; the radiance
 * cache is not available in batches.  1 <= n <= 4096,
 * fewer than 2^32 samples in all.  stats (nullable) receives the batch's
 * totals. */
int tet_render_batch(int32_t n, const tet_grid* const* grids, const tet_camera* cameras, const tet_medium* media,
                     const tet_light* lights, const int32_t* spp, const uint64_t* seeds,
                     const tet_render_opts* opts, float* const* out_rgb, void* hip_stream,
                     tet_render_stats* stats);

/* The same batch as a reusable frame: tet_batch_create fixes the scenes,
 * allocates the scratch memory and captures the frame's kernels in a HIP
 * graph; tet_batch_render replays it with new seeds (n values).  The grids
 * and output buffers must outlive the handle, and the grids' channels and
 * density models must not be replaced meanwhile (the frame reads them
 * where they were at creation). */
typedef struct tet_batch tet_batch;
int tet_batch_create(int32_t n, const tet_grid* const* grids, const tet_camera* cameras, const tet_medium* media,
                     const tet_light* lights, const int32_t* spp, const tet_render_opts* opts,
                     float* const* out_rgb, tet_batch** out);
int tet_batch_render(tet_batch* batch, const uint64_t* seeds, void* hip_stream, tet_render_stats* stats);
void tet_batch_free(tet_batch* batch);

/* Launch-option autotuner.  Times probe renders of the given frame (the
 * same camera at probe_spp samples per pixel) over the options that shape
 * scheduling only -- waves_per_simd, event_wait, batch_items, block_size,
 * record_layout; samples_per_item is set to 1 -- by coordinate descent from
 * `inout` (two sweeps, the
 * fastest of probe_repeats timings per candidate), and writes the fastest
 * into `inout`.  None of these options changes an image beyond FP32
 * summation order.  With a cache_path the result is looked up first and
 * stored after tuning, keyed by device, grid size (log2 of the tet count),
 * image size, max_bounces and transmittance; *best_ms (nullable) receives
 * the probe time of the chosen options (from the cache when found there). */
typedef struct {
  int32_t probe_spp;      /* samples per pixel of a probe render (default 2) */
  int32_t probe_repeats;  /* timings per candidate, fastest kept (default 2) */
  const char* cache_path; /* JSON cache file, or NULL */
} tet_autotune_opts;

void tet_autotune_opts_defaults(tet_autotune_opts* o);
int tet_autotune(const tet_grid* grid, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
                 const tet_autotune_opts* aopts /* NULL = defaults */, tet_render_opts* inout, void* hip_stream,
                 double* best_ms);

/* The face data of the traversal records as the walk reads them (paper,
 * "Path Tracing within Tetrahedral Grids": each face stored as one of 18
 * orientations and an offset, so an exit test is a few operations): per
 * tet and face f, codes[4 t + f] = 2 N + s (outward normal (-1)^s dir_N over
 * the 9 directions x, y, z, x+y, x-y, x+z, x-z, y+z, y-z), offsets[4 t + f] =
 * the outward normal . any vertex of the face, in lattice units (world *
 * 2^20), links[4 t + f] = the link word as stored.  layout 48: the 48-byte
 * records (link = (index << 2) | back face, or 0xFFFFFFFF on the boundary);
 * 32: the compact records (link = 27-bit index, or 2^27 - 1 on the
 * boundary; TET_ERR_INVALID_ARG when the grid has none).  Any output may be
 * NULL; all on one side (on_device). */
int tet_grid_export_faces(const tet_grid* grid, int32_t layout, uint8_t* codes, int32_t* offsets, uint32_t* links,
                          int32_t on_device, void* hip_stream);

/* Extra channels per tet (paper, "Volumetric Path Tracing": the
 * implementation also carries e.g. temperature, albedo and phase-function
 * parameters per tet).  Each given channel -- n^3 FP32 voxels, x fastest,
 * over the unit cube, n a power of two <= 4096 (independent of the density's
 * resolution) -- is reduced per tet to the mean over the voxels of the tet's
 * bounding box, the rule and summation order of the extinction.  temperature >= 0, albedo in [0, 1],
 * g in (-1, 1), else TET_ERR_NUMERIC and the grid is unchanged; NULL =
 * absent.  Replaces the grid's channels.  Buffers are the caller's. */
typedef struct {
  const float* temperature;
  const float* albedo;
  const float* g;
  int32_t n;
  int32_t on_device;
} tet_channels;

int tet_grid_set_channels(tet_grid* grid, const tet_channels* channels, void* hip_stream);
/* Per-tet values (num_tets each; NULL = skip; TET_ERR_INVALID_ARG for a
 * channel the grid does not have). */
int tet_grid_export_channels(const tet_grid* grid, float* temperature, float* albedo, float* g, int32_t on_device);

/* Density inside a tet (an extension of the paper's one density value per
 * tet, "Volumetric Path Tracing"; delta tracking against per-tet majorants
 * with true null collisions).  model:
 *   0  constant per tet (the build's extinction; density may be NULL);
 *   1  linear: the volume is sampled at each vertex by trilinear
 *      interpolation (values at voxel centres (i + 1/2) / n, indices clamped
 *      at the cube's faces; FP64, x then y then z) times density_scale, and
 *      interpolated linearly inside the tet, evaluated at a point as
 *      ((c0 + gx x) + gy y) + gz z in FP32 from per-tet coefficients
 *      rounded from FP64; majorant = the largest vertex value;
 *   2  voxel lookup: extinction at a point = density_scale * the voxel
 *      floor(x n) (indices clamped); majorant = density_scale * the largest
 *      voxel overlapping the tet's open bounding box.  The library keeps a
 *      device copy of the volume (n^3 * 4 bytes).
 * The volume is any n^3 FP32 grid (n a power of two <= 4096, values finite
 * and >= 0, else TET_ERR_NUMERIC and the grid unchanged), normally the one
 * the grid was built from; the caller's buffer is only read.  Renders of
 * the grid then use the model (each tentative collision evaluates the
 * extinction at its point; the analytic light transmittance of model 1
 * integrates it exactly per segment); model 2 needs ratio or delta
 * tracking for the light (transmittance 1 or 2, else TET_ERR_INVALID_ARG).
 * Both models render in batches and with a radiance cache, whose input
 * sigma at a vertex is then the model's extinction at the vertex.  Device
 * memory beyond the grid: copies of its
 * records carrying the model's majorant (48 bytes per tet, plus 32 with
 * compact records), 4 bytes per tet of majorant, and 16 bytes per tet of
 * coefficients (model 1) or the volume (model 2). */
int tet_grid_set_density_model(tet_grid* grid, const tet_density* density, int32_t model, void* hip_stream);
/* The model's per-tet majorant (num_tets floats) and, for model 1, the
 * coefficients (num_tets x {c0, gx, gy, gz}); NULL = skip.
 * TET_ERR_INVALID_ARG when the grid has no model (or coef for model 2). */
int tet_grid_export_density_model(const tet_grid* grid, float* majorant, float* coef, int32_t on_device);

/* Point location (the grid-entry step of Algorithm 1): canonical index of
 * the tet containing each point (3 FP32 per point, inside [0,1]^3), or -1.
 * pts and out live on the same side (on_device). */
int tet_locate(const tet_grid* grid, const float* pts, int64_t count, int64_t* out, int32_t on_device,
               void* hip_stream);

/* The tracer's elementary functions on the device, at n given arguments
 * (a test hook: their accuracy against the definitions they stand for).
 * Each is computed in FP64 and rounded once to FP32.  fn:
 *   0  -ln(1 - a), a in [0, 1)  (the exponential free path of Algorithm 1's
 *      free-path sampling, from a uniform);
 *   1  e^-a, a >= 0  (transmittance from an optical depth);
 *   2  (cos, sin)(2 pi a), a in [0, 1), written to out[2i], out[2i + 1]
 *      (the azimuth of a scattered direction);
 *   3  Henyey-Greenstein density of the cosine a for g = b[i];
 *   4  Henyey-Greenstein inverse CDF at a for g = b[i] (the cosine of a
 *      phase-function sample).
 * a, b (fn 3 and 4 only) and out (2n values for fn 2, else n) live on the
 * same side (on_device); n <= 2^30. */
int tet_eval_functions(int32_t fn, int64_t n, const float* a, const float* b, float* out, int32_t on_device,
                       void* hip_stream);

/* The same integrator on the regular voxel grid (the paper's regular-grid
 * reference renderer), voxels walked by Amanatides-Woo traversal. */
int dda_render(const tet_density* density, const tet_camera* camera, const tet_medium* medium,
               const tet_light* light, int32_t spp, uint64_t seed, const tet_render_opts* opts, float* out_rgb,
               int32_t on_device, void* hip_stream, tet_render_stats* stats);

void tet_grid_free(tet_grid* grid);

/* ---------------------------------------------------------------- radiance cache
 * A learned radiance cache (an addition to the paper's method, after
 * Mueller et al. 2021, "Real-time Neural Radiance Caching for Path
 * Tracing").  A small MLP maps a path vertex -- its position p, the
 * incoming direction d and the extinction sigma there (the cell's, or the
 * grid's density model at the vertex) --
 * to the radiance the rest of the path brings back per unit of throughput
 * reaching the vertex (before the vertex's albedo).  Rendering with a cache
 * (tet_render_opts.nrc) stops every path at real vertex truncate_bounce
 * and adds throughput x max(cache, 0) there; that vertex gets no light
 * estimate of its own (the cache covers it).  The cache learns online from
 * untruncated training paths of the scene (tet_nrc_train_frame).
 *
 * Network: 76 features -> 64 -> 64 -> 64 -> 64 -> 3, ReLU after hidden
 * layers, linear output; 17,603 parameters, stored layer by layer as W
 * (row-major [out][in]) then b.  Features: for axis a = x, y, z and
 * k = 0..11, sin(2^k pi p_a) at 24 a + 2 k and cos(2^k pi p_a) at
 * 24 a + 2 k + 1; then d (72..74) and log(1 + sigma) / log(1 + sigma_ref)
 * (75).  Products run on the matrix cores in BF16 with FP32 accumulation:
 * the weights, each layer's input and the back-propagated errors are
 * rounded to bfloat16 (nearest, ties to even); biases, bias gradients,
 * loss and Adam stay FP32, on FP32 master weights.  Loss: relative L2,
 * 1/(3B) sum (y - t)^2 / (y^2 + 0.01) with the denominator held constant.
 * Optimiser: Adam with bias correction.
 *
 * Training paths of a frame: path j < train_paths is the plain estimator's
 * sample j (Philox key frame_seed) of pixel floor(w (W H) / 2^24), w = the
 * upper 24 bits of word 0 of Philox(counter (j, 0, 4, 0)).  Each of its
 * real vertices k <= train_vertices with a positive throughput beta_k gives
 * a record (p, d, sigma, target = (L_final - L_before_k) / beta_k), in
 * (path, vertex) order. */

typedef struct {
  int32_t truncate_bounce;  /* real vertex at which rendering queries the cache, >= 1 (default 2) */
  int32_t train_paths;      /* training paths per frame, 1..2^24 (default 16384) */
  int32_t train_vertices;   /* vertices recorded per training path, 1..16 (default 4) */
  int32_t train_steps;      /* Adam steps per frame; the frame's records split in equal consecutive
                               batches (default 4) */
  float lr, beta1, beta2, eps; /* Adam (defaults 1e-3, 0.9, 0.99, 1e-8) */
  float sigma_ref;          /* extinction normaliser of the features, > 0; 0 = the largest extinction of
                               the first grid trained on (default 0) */
  float ema;                /* queries use the average ema_t = e ema_{t-1} + (1 - e) w_t of the weights
                               after each Adam step, divided by 1 - e^t (0 = the current weights;
                               default 0.95, 0 <= e < 1) */
  uint64_t seed;            /* weight initialisation (He-uniform weights, zero biases) */
} tet_nrc_opts;

typedef struct {
  int64_t records;  /* training records of the frame */
  double loss;      /* mean over the frame's Adam steps of the batch loss before the step */
  double ms;        /* device time of the call */
  double trace_ms;  /* of which tracing the training paths */
} tet_nrc_stats;

void tet_nrc_opts_defaults(tet_nrc_opts* o);
/* New cache on the current device; *out receives the handle. */
int tet_nrc_create(const tet_nrc_opts* opts /* NULL = defaults */, tet_nrc** out);
void tet_nrc_free(tet_nrc* nrc);
/* Options in force (sigma_ref resolved once set) and Adam steps taken. */
int tet_nrc_info(const tet_nrc* nrc, tet_nrc_opts* opts, int64_t* adam_steps);
/* FP32 master parameters out / in (17,603 values, layout above); import
 * also resets the Adam moments, the weight average and the step count.
 * tet_nrc_export_inference gives the weights queries use (the averaged
 * ones when ema > 0). */
int tet_nrc_export(const tet_nrc* nrc, float* params, int32_t on_device, void* hip_stream);
int tet_nrc_export_inference(const tet_nrc* nrc, float* params, int32_t on_device, void* hip_stream);
int tet_nrc_import(tet_nrc* nrc, const float* params, int32_t on_device, void* hip_stream);
/* Network outputs (unclamped) at `count` points: pos, dir count x 3,
 * sigma count (raw extinction), y count x 3; all on one side.  Needs
 * sigma_ref set. */
int tet_nrc_infer(const tet_nrc* nrc, int64_t count, const float* pos, const float* dir, const float* sigma,
                  float* y, int32_t on_device, void* hip_stream);
/* Gradient of sum_n dy_n . y_n over the parameters for explicit features
 * (count x 76 FP32) and output gradients dy (count x 3), with y; the cache
 * is not changed.  count <= 2^20.  grads: 17,603 values. */
int tet_nrc_forward_backward(const tet_nrc* nrc, int32_t count, const float* feats, const float* dy, float* y,
                             float* grads, int32_t on_device, void* hip_stream);
/* One Adam step on the relative-L2 loss of `count` records (count <= 2^20);
 * *loss (host, nullable) receives the batch loss before the step. */
int tet_nrc_train_batch(tet_nrc* nrc, int32_t count, const float* pos, const float* dir, const float* sigma,
                        const float* target, float* loss, int32_t on_device, void* hip_stream);
/* The training records of one frame (see above), without training:
 * capacity records at most (TET_ERR_CAPACITY beyond it, with *count set to
 * the number needed); tag = 16 j + (k - 1).  opts (nullable) gives
 * max_bounces, transmittance and max_steps_per_path of the paths. */
int tet_nrc_collect(const tet_nrc* nrc, const tet_grid* grid, const tet_camera* camera, const tet_medium* medium,
                    const tet_light* light, uint64_t frame_seed, const tet_render_opts* opts, float* pos, float* dir,
                    float* sigma, float* target, int32_t* tag, int64_t capacity, int64_t* count, int32_t on_device,
                    void* hip_stream);
/* Online training for one frame: trace the frame's training paths, then
 * train_steps Adam steps over their records. */
int tet_nrc_train_frame(tet_nrc* nrc, const tet_grid* grid, const tet_camera* camera, const tet_medium* medium,
                        const tet_light* light, uint64_t frame_seed, const tet_render_opts* opts, void* hip_stream,
                        tet_nrc_stats* stats /* nullable */);

/* Frees device memory cached by the library between calls: the blocks the
 * calling thread's calls released and those of threads that have ended
 * (each thread reuses only the blocks its own calls released, so calls on
 * different threads and streams never share scratch memory). */
void tet_release_cache(void);

const char* tet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
