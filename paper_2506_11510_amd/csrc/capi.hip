// capi.hip -- the extern "C" entry points of libtetvol.so, the host-side
// camera frames, the error state and the device-memory cache.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>

#include "nrc.h"

namespace tv {

int build_grid(const tet_density*, const tet_camera*, float, const tet_build_opts*, hipStream_t, tet_grid**);
int build_grid_sparse(const tet_sparse_density*, const tet_camera*, float, const tet_build_opts*, hipStream_t,
                      tet_grid**);
int grid_set_channels(tet_grid*, const tet_channels*, hipStream_t);
int grid_export_channels(const tet_grid*, float*, float*, float*, int32_t);
int grid_set_density_model(tet_grid*, const tet_density*, int32_t, hipStream_t);
int grid_export_density_model(const tet_grid*, float*, float*, int32_t);
int render_grid(const tet_grid*, const tet_camera*, const tet_medium*, const tet_light*, int32_t, uint64_t,
                const tet_render_opts*, float*, int32_t, hipStream_t, tet_render_stats*);
int render_voxels(const tet_density*, const tet_camera*, const tet_medium*, const tet_light*, int32_t, uint64_t,
                  const tet_render_opts*, float*, int32_t, hipStream_t, tet_render_stats*);
int locate_points(const tet_grid*, const float*, int64_t, int64_t*, int32_t, hipStream_t);
int eval_functions(int32_t, int64_t, const float*, const float*, float*, int32_t, hipStream_t);
int update_grid(tet_grid*, const tet_density*, const tet_camera*, float, const tet_build_opts*, hipStream_t);
int update_grid_sparse(tet_grid*, const tet_sparse_density*, const tet_camera*, float, const tet_build_opts*,
                       hipStream_t);
int render_grid_noalloc(const tet_grid*, const tet_camera*, const tet_medium*, const tet_light*, int32_t, uint64_t,
                        const tet_render_opts*, float*, hipStream_t);
int render_batch(int32_t, const tet_grid* const*, const tet_camera*, const tet_medium*, const tet_light*,
                 const int32_t*, const uint64_t*, const tet_render_opts*, float* const*, hipStream_t,
                 tet_render_stats*);
int batch_create(int32_t, const tet_grid* const*, const tet_camera*, const tet_medium*, const tet_light*,
                 const int32_t*, const tet_render_opts*, float* const*, void**);
int batch_render(void*, const uint64_t*, hipStream_t, tet_render_stats*);
void batch_free(void*);
int batch_device(const void*);
int autotune(const tet_grid*, const tet_camera*, const tet_medium*, const tet_light*, const tet_autotune_opts*,
             tet_render_opts*, hipStream_t, double*);

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

// ---------------------------------------------------------------- device memory cache
// Freed blocks are kept for reuse by the thread that freed them.  A call
// frees a block while its own kernels may still be queued on its stream;
// reuse in the same call is ordered on that stream, and by the time the call
// returns (calls are synchronous) the block is idle.  Another thread's call,
// on another stream, could otherwise take the block while those kernels
// still run.  Blocks of threads that have ended are idle and shared.
namespace {
using FreeList = std::multimap<std::pair<int, size_t>, void*>;  // (device, bytes) -> block
std::mutex g_mu;
FreeList g_idle;                                           // blocks of ended threads
std::unordered_map<void*, std::pair<int, size_t>> g_size;  // every block the cache made

struct ThreadBlocks {
  FreeList free;
  ~ThreadBlocks() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_idle.insert(free.begin(), free.end());
  }
};
thread_local ThreadBlocks t_blocks;

void* take(FreeList& fl, int dev, size_t bytes) {
  auto it = fl.lower_bound({dev, bytes});
  if (it == fl.end() || it->first.first != dev || it->first.second > 2 * bytes) return nullptr;
  void* p = it->second;
  fl.erase(it);
  return p;
}
}  // namespace

void* dev_alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (void* p = take(t_blocks.free, dev, bytes)) return p;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (void* p = take(g_idle, dev, bytes)) return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    tet_release_cache();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_size[p] = {dev, bytes};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  std::pair<int, size_t> key;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_size.find(p);
    if (it == g_size.end()) return;
    key = it->second;
  }
  t_blocks.free.insert({key, p});
}

// ---------------------------------------------------------------- cameras
static double dot3(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
static void unit3(double* v) {
  double l = std::sqrt(dot3(v, v));
  for (int i = 0; i < 3; i++) v[i] = v[i] / l;
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Orthonormal camera frame (forward, right, up) in FP64 from the FP32
// camera, and tan of the half fields of view.
static void frame64(const tet_camera& c, double pos[3], double f[3], double r[3], double u[3], double* tx,
                    double* ty) {
  double up[3];
  for (int i = 0; i < 3; i++) {
    pos[i] = (double)c.pos[i];
    f[i] = (double)c.look_at[i] - pos[i];
    up[i] = (double)c.up[i];
  }
  unit3(f);
  cross3(f, up, r);
  unit3(r);
  cross3(r, f, u);
  *ty = std::tan((double)c.fov_y_deg * (3.14159265358979323846 / 360.0));
  *tx = *ty * (double)c.width / (double)c.height;
}

void make_frame(const tet_camera& c, Frame* fr) {
  double pos[3], f[3], r[3], u[3], tx, ty;
  frame64(c, pos, f, r, u, &tx, &ty);
  for (int i = 0; i < 3; i++) {
    fr->pos[i] = c.pos[i];
    fr->f[i] = (float)f[i];
    fr->r[i] = (float)r[i];
    fr->u[i] = (float)u[i];
  }
  fr->tan_x = (float)tx;
  fr->tan_y = (float)ty;
  fr->w = c.width;
  fr->h = c.height;
}

void make_camcrit(const tet_camera& c, float target_px, CamCrit* cc) {
  double r[3], u[3], tx, ty;
  frame64(c, cc->pos, cc->f, r, u, &tx, &ty);
  double kpx = ((double)c.height * 0.5) / ty;
  for (int i = 0; i < 3; i++) {
    cc->side[0][i] = tx * cc->f[i] - r[i];
    cc->side[1][i] = tx * cc->f[i] + r[i];
    cc->side[2][i] = ty * cc->f[i] - u[i];
    cc->side[3][i] = ty * cc->f[i] + u[i];
  }
  for (int s = 0; s < 4; s++) unit3(cc->side[s]);
  cc->kpx2 = kpx * kpx;
  cc->tgt2 = (double)target_px * (double)target_px;
}

int check_camera(const tet_camera* c) {
  if (!c) return fail(TET_ERR_INVALID_ARG, "camera is NULL");
  if (c->width < 1 || c->height < 1 || c->width > 65536 || c->height > 65536)
    return fail(TET_ERR_INVALID_ARG, "camera: width and height must be in [1, 65536]");
  if (!(c->fov_y_deg > 0.0f && c->fov_y_deg < 180.0f)) return fail(TET_ERR_INVALID_ARG, "camera: fov_y_deg must be in (0, 180)");
  double f[3], up[3], x[3];
  for (int i = 0; i < 3; i++) {
    if (!std::isfinite(c->pos[i]) || !std::isfinite(c->look_at[i]) || !std::isfinite(c->up[i]))
      return fail(TET_ERR_INVALID_ARG, "camera: non-finite vector");
    f[i] = (double)c->look_at[i] - (double)c->pos[i];
    up[i] = c->up[i];
  }
  cross3(f, up, x);
  if (!(dot3(f, f) > 0.0) || !(dot3(x, x) > 0.0))
    return fail(TET_ERR_INVALID_ARG, "camera: look_at equals pos or up is parallel to the view direction");
  return TET_OK;
}

// ---------------------------------------------------------------- export kernels
__global__ void k_export(int64_t n, const uint64_t* __restrict__ verts, const TetRec* __restrict__ rec,
                         uint32_t* __restrict__ nbr4, float* __restrict__ sigma, float* __restrict__ maj,
                         int32_t* __restrict__ v12) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  TetRec r = rec[i];
  if (nbr4)
    for (int f = 0; f < 4; f++) nbr4[4 * i + f] = r.nbr[f];
  if (sigma) sigma[i] = r.sigma;
  if (maj) maj[i] = r.majorant;
  if (v12)
    for (int j = 0; j < 4; j++) {
      uint64_t p = verts[4 * i + j];
      v12[12 * i + 3 * j] = vx(p);
      v12[12 * i + 3 * j + 1] = vy(p);
      v12[12 * i + 3 * j + 2] = vz(p);
    }
}

static int export_grid(const tet_grid* g, uint64_t* ids, uint32_t* nbr4, float* sigma, float* maj, int32_t* v12,
                       int32_t on_device, hipStream_t st) {
  int64_t n = g->n;
  size_t b_ids = n * 8, b_nbr = n * 16, b_s = n * 4, b_v = n * 48;
  char* tmp = nullptr;
  uint64_t* d_ids = ids;
  uint32_t* d_nbr = nbr4;
  float *d_s = sigma, *d_m = maj;
  int32_t* d_v = v12;
  if (!on_device) {
    size_t tot = (ids ? b_ids : 0) + (nbr4 ? b_nbr : 0) + (sigma ? b_s : 0) + (maj ? b_s : 0) + (v12 ? b_v : 0);
    tmp = (char*)dev_alloc(tot + 64);
    if (!tmp) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_export: scratch");
    char* q = tmp;
    if (ids) { d_ids = (uint64_t*)q; q += b_ids; }
    if (nbr4) { d_nbr = (uint32_t*)q; q += b_nbr; }
    if (sigma) { d_s = (float*)q; q += b_s; }
    if (maj) { d_m = (float*)q; q += b_s; }
    if (v12) { d_v = (int32_t*)q; q += b_v; }
  }
  struct Free {
    void* p;
    ~Free() { if (p) dev_free(p); }
  } f_{tmp};
  if (ids) TV_HIP(hipMemcpyAsync(d_ids, g->ids, b_ids, hipMemcpyDeviceToDevice, st));
  if (nbr4 || sigma || maj || v12) {
    hipLaunchKernelGGL(k_export, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, g->verts, g->rec, d_nbr,
                       d_s, d_m, d_v);
    TV_HIP(hipGetLastError());
  }
  if (!on_device) {
    if (ids) TV_HIP(hipMemcpyAsync(ids, d_ids, b_ids, hipMemcpyDeviceToHost, st));
    if (nbr4) TV_HIP(hipMemcpyAsync(nbr4, d_nbr, b_nbr, hipMemcpyDeviceToHost, st));
    if (sigma) TV_HIP(hipMemcpyAsync(sigma, d_s, b_s, hipMemcpyDeviceToHost, st));
    if (maj) TV_HIP(hipMemcpyAsync(maj, d_m, b_s, hipMemcpyDeviceToHost, st));
    if (v12) TV_HIP(hipMemcpyAsync(v12, d_v, b_v, hipMemcpyDeviceToHost, st));
  }
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

// Face data of the traversal records as stored: per face the orientation
// code, the plane offset in lattice units and the link word.
__global__ void k_export_faces(int64_t n, const TetRec* __restrict__ rec, const TetRec32* __restrict__ rec32,
                               uint8_t* __restrict__ codes, int32_t* __restrict__ offs,
                               uint32_t* __restrict__ links) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (rec32) {
    const TetRec32 r = rec32[i];
    const uint32_t o1 = (uint32_t)((((uint64_t)r.w[1] << 32) | r.w[0]) >> 23);
    const uint32_t o2 = (uint32_t)((((uint64_t)r.w[2] << 32) | r.w[1]) >> 14);
    const int32_t io[4] = {((int32_t)(r.w[0] << 9)) >> 9, ((int32_t)(o1 << 9)) >> 9, ((int32_t)(o2 << 9)) >> 9,
                           ((int32_t)(r.w[2] << 4)) >> 9};
    for (int f = 0; f < 4; f++) {
      if (codes) codes[4 * i + f] = (uint8_t)code_of32(r.w[4 + f]);
      if (offs) offs[4 * i + f] = io[f];
      if (links) links[4 * i + f] = r.w[4 + f] & kLink27Boundary;
    }
  } else {
    const TetRec r = rec[i];
    for (int f = 0; f < 4; f++) {
      if (codes) codes[4 * i + f] = (uint8_t)((r.codes >> (8 * f)) & 0xFFu);
      if (offs) offs[4 * i + f] = (int32_t)(r.off[f] * 0x1p20f);  // n_f . v * 2^-20, exact
      if (links) links[4 * i + f] = r.nbr[f];
    }
  }
}

static int export_faces(const tet_grid* g, int32_t layout, uint8_t* codes, int32_t* offs, uint32_t* links,
                        int32_t on_device, hipStream_t st) {
  if (!g || (layout != 32 && layout != 48)) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_faces: bad arguments");
  if (layout == 32 && !g->rec32) return fail(TET_ERR_INVALID_ARG, "tet_grid_export_faces: no compact records");
  const int64_t n = g->n;
  const size_t b_c = (size_t)n * 4, b_o = (size_t)n * 16;
  uint8_t* d_c = codes;
  int32_t* d_o = offs;
  uint32_t* d_l = links;
  char* tmp = nullptr;
  if (!on_device) {
    tmp = (char*)dev_alloc((codes ? b_c : 0) + (offs ? b_o : 0) + (links ? b_o : 0) + 64);
    if (!tmp) return fail(TET_ERR_OUT_OF_MEMORY, "tet_grid_export_faces: scratch");
    char* q = tmp;
    if (offs) { d_o = (int32_t*)q; q += b_o; }
    if (links) { d_l = (uint32_t*)q; q += b_o; }
    if (codes) d_c = (uint8_t*)q;
  }
  struct Free {
    void* p;
    ~Free() { if (p) dev_free(p); }
  } f_{tmp};
  if (codes || offs || links) {
    hipLaunchKernelGGL(k_export_faces, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, g->rec,
                       layout == 32 ? g->rec32 : nullptr, d_c, d_o, d_l);
    TV_HIP(hipGetLastError());
  }
  if (!on_device) {
    if (codes) TV_HIP(hipMemcpyAsync(codes, d_c, b_c, hipMemcpyDeviceToHost, st));
    if (offs) TV_HIP(hipMemcpyAsync(offs, d_o, b_o, hipMemcpyDeviceToHost, st));
    if (links) TV_HIP(hipMemcpyAsync(links, d_l, b_o, hipMemcpyDeviceToHost, st));
  }
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

}  // namespace tv

using namespace tv;

#define TV_GUARD(expr)                                      \
  try {                                                     \
    return (expr);                                          \
  } catch (const std::exception& e) {                       \
    return fail(TET_ERR_INTERNAL, e.what());                \
  } catch (...) {                                           \
    return fail(TET_ERR_INTERNAL, "unknown exception");     \
  }

extern "C" {

void tet_build_opts_defaults(tet_build_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->want_mode = 0;
  o->uniform_depth = 9;
  o->max_depth = 24;
  o->majorant_mode = 0;
  o->variation_tau = 0.2;
  o->max_tets = 1ll << 26;
}

void tet_render_opts_defaults(tet_render_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->max_bounces = 32;
  o->transmittance = 0;
  o->max_steps_per_path = 0x7FFFFFFF;
}

int leb_build(const tet_density* density, const tet_camera* camera, float target_cell_px, const tet_build_opts* opts,
              void* hip_stream, tet_grid** out) {
  TV_GUARD(build_grid(density, camera, target_cell_px, opts, (hipStream_t)hip_stream, out));
}

int leb_build_sparse(const tet_sparse_density* density, const tet_camera* camera, float target_cell_px,
                     const tet_build_opts* opts, void* hip_stream, tet_grid** out) {
  TV_GUARD(build_grid_sparse(density, camera, target_cell_px, opts, (hipStream_t)hip_stream, out));
}

int leb_update(tet_grid* grid, const tet_density* density, const tet_camera* camera, float target_cell_px,
               const tet_build_opts* opts, void* hip_stream) {
  TV_GUARD(update_grid(grid, density, camera, target_cell_px, opts, (hipStream_t)hip_stream));
}

int leb_update_sparse(tet_grid* grid, const tet_sparse_density* density, const tet_camera* camera,
                      float target_cell_px, const tet_build_opts* opts, void* hip_stream) {
  TV_GUARD(update_grid_sparse(grid, density, camera, target_cell_px, opts, (hipStream_t)hip_stream));
}

int tet_grid_info(const tet_grid* g, int64_t* num_tets, int32_t* max_depth, tet_build_stats* stats) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_grid_info: grid is NULL");
  if (num_tets) *num_tets = g->n;
  if (max_depth) *max_depth = g->max_depth;
  if (stats) *stats = g->stats;
  return TET_OK;
}

int tet_grid_export(const tet_grid* g, uint64_t* ids, uint32_t* nbr4, float* sigma, float* majorant, int32_t* verts12,
                    int32_t on_device, void* hip_stream) {
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_grid_export: grid is NULL");
  TV_GUARD(export_grid(g, ids, nbr4, sigma, majorant, verts12, on_device, (hipStream_t)hip_stream));
}

int tet_grid_set_channels(tet_grid* g, const tet_channels* channels, void* hip_stream) {
  TV_GUARD(grid_set_channels(g, channels, (hipStream_t)hip_stream));
}

int tet_grid_export_channels(const tet_grid* g, float* temperature, float* albedo, float* gch, int32_t on_device) {
  TV_GUARD(grid_export_channels(g, temperature, albedo, gch, on_device));
}

int tet_grid_set_density_model(tet_grid* g, const tet_density* density, int32_t model, void* hip_stream) {
  TV_GUARD(grid_set_density_model(g, density, model, (hipStream_t)hip_stream));
}

int tet_grid_export_density_model(const tet_grid* g, float* majorant, float* coef, int32_t on_device) {
  TV_GUARD(grid_export_density_model(g, majorant, coef, on_device));
}

int tet_render(const tet_grid* g, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
               int32_t spp, uint64_t seed, const tet_render_opts* opts, float* out_rgb, int32_t on_device,
               void* hip_stream, tet_render_stats* stats) {
  TV_GUARD(render_grid(g, camera, medium, light, spp, seed, opts, out_rgb, on_device, (hipStream_t)hip_stream, stats));
}

int tet_locate(const tet_grid* g, const float* pts, int64_t count, int64_t* out, int32_t on_device, void* hip_stream) {
  TV_GUARD(locate_points(g, pts, count, out, on_device, (hipStream_t)hip_stream));
}

int tet_grid_export_faces(const tet_grid* grid, int32_t layout, uint8_t* codes, int32_t* offsets, uint32_t* links,
                          int32_t on_device, void* hip_stream) {
  TV_GUARD(export_faces(grid, layout, codes, offsets, links, on_device, (hipStream_t)hip_stream));
}

int tet_render_noalloc(const tet_grid* g, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
                       int32_t spp, uint64_t seed, const tet_render_opts* opts, float* out_rgb, void* hip_stream) {
  TV_GUARD(render_grid_noalloc(g, camera, medium, light, spp, seed, opts, out_rgb, (hipStream_t)hip_stream));
}

int tet_eval_functions(int32_t fn, int64_t n, const float* a, const float* b, float* out, int32_t on_device,
                       void* hip_stream) {
  TV_GUARD(eval_functions(fn, n, a, b, out, on_device, (hipStream_t)hip_stream));
}

int dda_render(const tet_density* density, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
               int32_t spp, uint64_t seed, const tet_render_opts* opts, float* out_rgb, int32_t on_device,
               void* hip_stream, tet_render_stats* stats) {
  TV_GUARD(render_voxels(density, camera, medium, light, spp, seed, opts, out_rgb, on_device, (hipStream_t)hip_stream,
                         stats));
}

void tet_grid_free(tet_grid* g) {
  if (!g) return;
  dev_free(g->ids);
  dev_free(g->keys);
  dev_free(g->kidx);
  dev_free(g->verts);
  dev_free(g->chain);
  dev_free(g->rec);
  dev_free(g->rec32);
  for (int k = 0; k < 3; k++) dev_free(g->ch[k]);
  dev_free(g->mmaj);
  dev_free(g->mcoef);
  dev_free(g->mdens);
  dev_free(g->mrec);
  dev_free(g->mrec32);
  delete g;
}

void tet_release_cache(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (FreeList* fl : {&t_blocks.free, &g_idle}) {
    for (auto it = fl->begin(); it != fl->end();) {
      (void)hipSetDevice(it->first.first);
      (void)hipFree(it->second);
      g_size.erase(it->second);
      it = fl->erase(it);
    }
  }
  (void)hipSetDevice(cur);
}

void tet_autotune_opts_defaults(tet_autotune_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->probe_spp = 2;
  o->probe_repeats = 2;
  o->cache_path = nullptr;
}

int tet_autotune(const tet_grid* grid, const tet_camera* camera, const tet_medium* medium, const tet_light* light,
                 const tet_autotune_opts* aopts, tet_render_opts* inout, void* hip_stream, double* best_ms) {
  TV_GUARD(autotune(grid, camera, medium, light, aopts, inout, (hipStream_t)hip_stream, best_ms));
}

int tet_render_batch(int32_t n, const tet_grid* const* grids, const tet_camera* cameras, const tet_medium* media,
                     const tet_light* lights, const int32_t* spp, const uint64_t* seeds,
                     const tet_render_opts* opts, float* const* out_rgb, void* hip_stream,
                     tet_render_stats* stats) {
  TV_GUARD(render_batch(n, grids, cameras, media, lights, spp, seeds, opts, out_rgb, (hipStream_t)hip_stream, stats));
}

int tet_batch_create(int32_t n, const tet_grid* const* grids, const tet_camera* cameras, const tet_medium* media,
                     const tet_light* lights, const int32_t* spp, const tet_render_opts* opts,
                     float* const* out_rgb, tet_batch** out) {
  TV_GUARD(batch_create(n, grids, cameras, media, lights, spp, opts, out_rgb, (void**)out));
}

int tet_batch_render(tet_batch* batch, const uint64_t* seeds, void* hip_stream, tet_render_stats* stats) {
  TV_GUARD(batch_render(batch, seeds, (hipStream_t)hip_stream, stats));
}

void tet_batch_free(tet_batch* batch) {
  if (!batch) return;
  int cur = 0, dev = batch_device(batch);
  bool sw = hipGetDevice(&cur) == hipSuccess && cur != dev && hipSetDevice(dev) == hipSuccess;
  batch_free(batch);
  if (sw) (void)hipSetDevice(cur);
}

void tet_nrc_opts_defaults(tet_nrc_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->truncate_bounce = 2;
  o->train_paths = 16384;
  o->train_vertices = 4;
  o->train_steps = 4;
  o->lr = 1e-3f;
  o->beta1 = 0.9f;
  o->beta2 = 0.99f;
  o->eps = 1e-8f;
  o->sigma_ref = 0.0f;
  o->ema = 0.95f;
  o->seed = 0x5EEDull;
}

int tet_nrc_create(const tet_nrc_opts* opts, tet_nrc** out) { TV_GUARD(nrc_create(opts, out)); }

void tet_nrc_free(tet_nrc* nrc) {
  if (!nrc) return;
  int cur = 0;
  bool sw = hipGetDevice(&cur) == hipSuccess && cur != nrc->device && hipSetDevice(nrc->device) == hipSuccess;
  nrc_free(nrc);
  if (sw) (void)hipSetDevice(cur);
}

int tet_nrc_info(const tet_nrc* nrc, tet_nrc_opts* opts, int64_t* adam_steps) {
  if (!nrc) return fail(TET_ERR_INVALID_ARG, "tet_nrc_info: cache is NULL");
  if (opts) *opts = nrc->opts;
  if (adam_steps) *adam_steps = nrc->step;
  return TET_OK;
}

int tet_nrc_export(const tet_nrc* nrc, float* params, int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_export(nrc, params, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_export_inference(const tet_nrc* nrc, float* params, int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_export_inference(nrc, params, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_import(tet_nrc* nrc, const float* params, int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_import(nrc, params, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_infer(const tet_nrc* nrc, int64_t count, const float* pos, const float* dir, const float* sigma, float* y,
                  int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_infer(nrc, count, pos, dir, sigma, y, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_forward_backward(const tet_nrc* nrc, int32_t count, const float* feats, const float* dy, float* y,
                             float* grads, int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_forward_backward(nrc, count, feats, dy, y, grads, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_train_batch(tet_nrc* nrc, int32_t count, const float* pos, const float* dir, const float* sigma,
                        const float* target, float* loss, int32_t on_device, void* hip_stream) {
  TV_GUARD(nrc_train_batch(nrc, count, pos, dir, sigma, target, loss, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_collect(const tet_nrc* nrc, const tet_grid* grid, const tet_camera* camera, const tet_medium* medium,
                    const tet_light* light, uint64_t frame_seed, const tet_render_opts* opts, float* pos, float* dir,
                    float* sigma, float* target, int32_t* tag, int64_t capacity, int64_t* count, int32_t on_device,
                    void* hip_stream) {
  TV_GUARD(nrc_collect(nrc, grid, camera, medium, light, frame_seed, opts, pos, dir, sigma, target, tag, capacity,
                       count, on_device, (hipStream_t)hip_stream));
}

int tet_nrc_train_frame(tet_nrc* nrc, const tet_grid* grid, const tet_camera* camera, const tet_medium* medium,
                        const tet_light* light, uint64_t frame_seed, const tet_render_opts* opts, void* hip_stream,
                        tet_nrc_stats* stats) {
  TV_GUARD(nrc_train_frame(nrc, grid, camera, medium, light, frame_seed, opts, (hipStream_t)hip_stream, stats));
}

const char* tet_last_error(void) { return g_err.c_str(); }

}  // extern "C"
