// nrc.h -- the learned radiance cache's device state and the calls the
// tracer and the cache make into each other (internal to libtetvol).
#pragma once
#include "common.h"

namespace tv {

// Network 76 -> 64 -> 64 -> 64 -> 64 -> 3; parameters layer by layer, W
// row-major [out][in] then b.
constexpr int kNrcIn = 76;
constexpr int kNrcParams = 17603;
__host__ __device__ constexpr int nrc_off_w(int l) { return l == 0 ? 0 : 4928 + (l - 1) * 4160; }
__host__ __device__ constexpr int nrc_off_b(int l) { return l == 0 ? 4864 : (l < 4 ? nrc_off_w(l) + 4096 : 17600); }
static_assert(nrc_off_b(4) + 3 == kNrcParams, "parameter count");

// Packed network for the matrix cores: 66 operand fragments of 1 KiB (64
// lanes x 8 bfloat16) -- 38 for the forward products, 28 for the
// transposed products of the backward pass -- then 272 FP32 biases (4 x 64
// hidden, the output's 3 padded to 16).
constexpr int kNrcFrags = 66;
constexpr int kNrcFwdFrags = 38;
constexpr int kNrcBias = 272;
constexpr size_t kNrcNetBytes = (size_t)kNrcFrags * 1024 + (size_t)kNrcBias * 4;

// The cache queries of a render pass: *qcount compacted queries of 32
// bytes, (x, y, z, sigma), (dx, dy, dz, beta), and their pixels; each adds
// beta * max(cache, 0) to its pixel's running sum in `out` (atomically).
// capacity bounds *qcount.
int nrc_query_pass(const tet_nrc* nrc, const float4* q, const uint32_t* qpix, const uint32_t* qcount, float* out,
                   int64_t capacity, hipStream_t st);

// Traces the training paths of a frame (untruncated), writing per path up
// to kv vertex records of 3 float4 -- (x, sigma), (d, beta before the
// albedo), (L gathered before the vertex, 0) -- at vrec[(j kv + k) 3], and
// (L_final, real vertex count as a float's bits) at path_l[j].
int trace_training_paths(const tet_grid* g, const tet_camera* cam, const tet_medium* med, const tet_light* light,
                         uint64_t frame_seed, const tet_render_opts* opts, int32_t n_paths, int32_t kv, float4* vrec,
                         float4* path_l, hipStream_t st, float* ms);

// Compaction of training paths a render traced and the cache's Adam steps
// on their records (nrc.hip); *records, *loss (nullable) report them.
int nrc_train_paths(tet_nrc* n, const float4* vrec, const float4* path_l, int32_t n_paths, int32_t kv, hipStream_t st,
                    int64_t* records, double* loss);
// sigma_ref from the grid's largest extinction when it is not set yet.
int nrc_resolve_sigma_ref(tet_nrc* n, const tet_grid* g, hipStream_t st);

// Host side of the C ABI (nrc.hip).
int nrc_create(const tet_nrc_opts* opts, tet_nrc** out);
void nrc_free(tet_nrc* n);
int nrc_export(const tet_nrc* n, float* params, int32_t on_device, hipStream_t st);
int nrc_import(tet_nrc* n, const float* params, int32_t on_device, hipStream_t st);
int nrc_export_inference(const tet_nrc* n, float* params, int32_t on_device, hipStream_t st);
int nrc_infer(const tet_nrc* n, int64_t count, const float* pos, const float* dir, const float* sigma, float* y,
              int32_t on_device, hipStream_t st);
int nrc_forward_backward(const tet_nrc* n, int32_t count, const float* feats, const float* dy, float* y, float* grads,
                         int32_t on_device, hipStream_t st);
int nrc_train_batch(tet_nrc* n, int32_t count, const float* pos, const float* dir, const float* sigma,
                    const float* target, float* loss, int32_t on_device, hipStream_t st);
int nrc_collect(const tet_nrc* n, const tet_grid* g, const tet_camera* cam, const tet_medium* med,
                const tet_light* light, uint64_t frame_seed, const tet_render_opts* ro, float* pos, float* dir,
                float* sigma, float* target, int32_t* tag, int64_t capacity, int64_t* count, int32_t on_device,
                hipStream_t st);
int nrc_train_frame(tet_nrc* n, const tet_grid* g, const tet_camera* cam, const tet_medium* med,
                    const tet_light* light, uint64_t frame_seed, const tet_render_opts* ro, hipStream_t st,
                    tet_nrc_stats* stats);

}  // namespace tv

struct tet_nrc {
  int device;
  tet_nrc_opts opts;
  int64_t step;    // Adam steps taken
  float* master;   // FP32 parameters
  float* m;        // Adam first moments
  float* v;        // Adam second moments
  char* net;       // packed network of the master weights (training)
  float* ema;      // weight average (zero-initialised)
  float* infer;    // the weights queries use: ema / (1 - e^step), or the master weights
  char* net_infer; // packed network of `infer`
  // packed network the queries use
  const char* query_net() const { return opts.ema > 0.0f ? net_infer : net; }
};
