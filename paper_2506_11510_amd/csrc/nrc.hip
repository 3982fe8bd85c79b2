// nrc.hip -- the learned radiance cache (an addition to the paper's method,
// after Mueller et al. 2021): feature encoding, the MLP on the matrix cores,
// relative-L2 loss, backward pass and Adam, and the cache's host calls.
//
// Matrix-core layout.  One wave evaluates 64 samples as 4 column blocks of
// 16.  Every product is taken transposed, Y^T = W X^T, with
// v_mfma_f32_16x16x32_bf16 (D[16x16] += A[16x32] B[32x16], FP32
// accumulation): A is a 16-row block of W, B a 32-deep slice of the layer
// input for 16 samples.  Lane l (r = l % 16, g = l / 16) holds A row r and
// B column r (one sample) at k = 8g..8g+7, and D rows 4g..4g+3 of column r.
// So after a layer, lane l holds 4 consecutive units of one sample in each
// 16-unit block; the next layer's B operand for k-slice ks takes them from
// the D blocks 2ks and 2ks+1, i.e. its k order is
//   kmap(ks, g, e) = 32 ks + 16 (e / 4) + 4 g + e % 4,
// and every later layer's weight fragments are stored with their input
// index permuted the same way.  Activations stay in registers from layer to
// layer.  Backward, errors propagate the same way through fragments of the
// transposed weights; dW = delta a^T contracts over samples, so the layer
// inputs and errors are also kept in LDS as [unit][sample] rows, from which
// either operand's 8 consecutive samples are one 16-byte read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nrc.h"

namespace tv {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline u32x4 as_u4(bf16x8 v) { return __builtin_bit_cast(u32x4, v); }

// bfloat16 bits of a finite x, rounded to nearest, ties to even.
__device__ inline uint32_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline uint32_t pack2(float a, float b) { return bf16_rne(a) | (bf16_rne(b) << 16); }
__device__ inline bool bf16_positive(uint16_t h) { return __uint_as_float((uint32_t)h << 16) > 0.0f; }

__host__ __device__ constexpr int kmap(int ks, int g, int e) { return 32 * ks + 16 * (e >> 2) + 4 * g + (e & 3); }

// Fragment bases (in 1 KiB fragments): forward W0 [rb][ks<3], W1..W3
// [rb][ks<2], W4 [ks<2]; backward W4^T [rb], W3^T, W2^T, W1^T [rb][ks<2].
constexpr int kF0 = 0, kF1 = 12, kF2 = 20, kF3 = 28, kF4 = 36, kB4 = 38, kB3 = 42, kB2 = 50, kB1 = 58;
__host__ __device__ constexpr int frag_fwd(int l) { return l == 0 ? kF0 : 12 + 8 * (l - 1); }
__host__ __device__ constexpr int frag_bwd(int l) { return l == 4 ? kB4 : 42 + 8 * (3 - l); }
static_assert(frag_fwd(4) == kF4 && frag_bwd(3) == kB3 && frag_bwd(1) == kB1, "fragment map");

// Element e of lane l of fragment f, from the FP32 parameters P.
__device__ inline float frag_value(const float* P, int f, int l, int e) {
  const int r = l & 15, g = l >> 4;
  if (f < kF1) {  // W0: row 16 rb + r, natural input order (76 inputs, zero beyond)
    int o = 16 * (f / 3) + r, i = 32 * (f % 3) + 8 * g + e;
    return i < kNrcIn ? P[nrc_off_w(0) + o * kNrcIn + i] : 0.0f;
  }
  if (f < kF4) {  // W1..W3
    int L = 1 + (f - kF1) / 8, q = (f - kF1) % 8;
    return P[nrc_off_w(L) + (16 * (q / 2) + r) * 64 + kmap(q % 2, g, e)];
  }
  if (f < kB4) {  // W4: rows = the 3 outputs, padded to 16
    return r < 3 ? P[nrc_off_w(4) + r * 64 + kmap(f - kF4, g, e)] : 0.0f;
  }
  if (f < kB3) {  // W4^T: row = input unit 16 rb + r, k = output kmap(0, g, e) (3 of them)
    int o = kmap(0, g, e);
    return o < 3 ? P[nrc_off_w(4) + o * 64 + 16 * (f - kB4) + r] : 0.0f;
  }
  int q = f - kB3, L = 3 - q / 8;  // W3^T, W2^T, W1^T
  q %= 8;
  return P[nrc_off_w(L) + kmap(q % 2, g, e) * 64 + 16 * (q / 2) + r];
}

// FP32 parameters -> packed network (fragments, then the biases).
__global__ void k_nrc_pack(const float* __restrict__ P, char* __restrict__ net) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int kWords = kNrcFrags * 256;
  if (t < kWords) {
    int f = t >> 8, l = (t >> 2) & 63, w = t & 3;
    ((uint32_t*)net)[t] = pack2(frag_value(P, f, l, 2 * w), frag_value(P, f, l, 2 * w + 1));
  } else if (t < kWords + kNrcBias) {
    int b = t - kWords;
    float v = b < 256 ? P[nrc_off_b(b >> 6) + (b & 63)] : (b - 256 < 3 ? P[nrc_off_b(4) + b - 256] : 0.0f);
    ((float*)(net + kNrcFrags * 1024))[b] = v;
  }
}

// ---------------------------------------------------------------- encoding
// Features 8c..8c+7 (c = 0..11) of one sample: sin / cos (2^k pi p_a) for
// c < 9 (axis c / 3, k = 4 (c % 3) .. +3), then d and the normalised
// extinction, then zeros.  2^k p is exact, and so is its reduction modulo 2,
// r; sin / cos (pi r) = sin / cos (2 pi (r / 2)).
__device__ inline bf16x8 feat_chunk(int c, float px, float py, float pz, float dx, float dy, float dz, float sigma,
                                    double lref) {
  u32x4 v = {0u, 0u, 0u, 0u};
  if (c < 9) {
    float x = c < 3 ? px : (c < 6 ? py : pz);
    int k0 = 4 * (c % 3);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      float y = ldexpf(x, k0 + j);
      float r = y - 2.0f * floorf(y * 0.5f);
      float cs, sn;
      sincos_2pi(r * 0.5f, cs, sn);
      v[j] = pack2(sn, cs);
    }
  } else if (c == 9) {
    float sn = (float)(log1p((double)sigma) / lref);
    v[0] = pack2(dx, dy);
    v[1] = pack2(dz, sn);
  }
  return as_bf(v);
}

__device__ inline bf16x8 feat_chunk_mem(const float* f, int c) {
  u32x4 v;
#pragma unroll
  for (int w = 0; w < 4; w++) {
    int i = 8 * c + 2 * w;
    v[w] = pack2(i < kNrcIn ? f[i] : 0.0f, i + 1 < kNrcIn ? f[i + 1] : 0.0f);
  }
  return as_bf(v);
}

// ---------------------------------------------------------------- layers
// acc[rb][cb] = b + W x over KS k-slices; F = the layer's fragments [rb][ks].
template <int KS>
__device__ inline void layer_fwd(const u32x4* F, const float* bias, const bf16x8 (&X)[4][KS], f32x4 (&acc)[4][4],
                                 int lane) {
  const int g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < 4; rb++) {
    f32x4 b = *(const f32x4*)(bias + 16 * rb + 4 * g);
#pragma unroll
    for (int cb = 0; cb < 4; cb++) acc[rb][cb] = b;
  }
#pragma unroll
  for (int ks = 0; ks < KS; ks++)
#pragma unroll
    for (int rb = 0; rb < 4; rb++) {
      bf16x8 a = as_bf(F[(rb * KS + ks) * 64 + lane]);
#pragma unroll
      for (int cb = 0; cb < 4; cb++) acc[rb][cb] = mfma(a, X[cb][ks], acc[rb][cb]);
    }
}

// Next layer's B operand (k order kmap) from D blocks 2ks, 2ks + 1.
template <bool RELU>
__device__ inline bf16x8 dpack(f32x4 lo, f32x4 hi) {
  if (RELU) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      lo[i] = fmaxf(lo[i], 0.0f);
      hi[i] = fmaxf(hi[i], 0.0f);
    }
  }
  u32x4 v = {pack2(lo[0], lo[1]), pack2(lo[2], lo[3]), pack2(hi[0], hi[1]), pack2(hi[2], hi[3])};
  return as_bf(v);
}

template <bool RELU>
__device__ inline void to_operand(const f32x4 (&acc)[4][4], bf16x8 (&H)[4][2]) {
#pragma unroll
  for (int cb = 0; cb < 4; cb++)
#pragma unroll
    for (int ks = 0; ks < 2; ks++) H[cb][ks] = dpack<RELU>(acc[2 * ks][cb], acc[2 * ks + 1][cb]);
}

__device__ inline void out_fwd(const u32x4* F4, const float* bias4, const bf16x8 (&H)[4][2], f32x4 (&o)[4],
                               int lane) {
  f32x4 b = *(const f32x4*)(bias4 + 4 * (lane >> 4));
#pragma unroll
  for (int cb = 0; cb < 4; cb++) o[cb] = b;
#pragma unroll
  for (int ks = 0; ks < 2; ks++) {
    bf16x8 a = as_bf(F4[ks * 64 + lane]);
#pragma unroll
    for (int cb = 0; cb < 4; cb++) o[cb] = mfma(a, H[cb][ks], o[cb]);
  }
}

// ---------------------------------------------------------------- query
struct NrcQueryArgs {
  const char* net;
  double lref;  // log(1 + sigma_ref)
  int64_t count;
  const float* pos;  // mode 0: inputs (count x 3, x 3, x 1) and raw outputs (count x 3)
  const float* dir;
  const float* sigma;
  float* y;
  const float4* q;          // mode 1: compacted query records, their pixels, their number
  const uint32_t* qpix;
  const uint32_t* qcount;
  float* out;               // running pixel sums
};

// Mode 0: network outputs at explicit points.  Mode 1: a render pass's
// queries; each adds beta * max(y, 0) to its pixel.
template <int MODE>
__global__ __launch_bounds__(256) void k_nrc_query(NrcQueryArgs Q) {
  __shared__ u32x4 s_frag[kNrcFwdFrags * 64];
  __shared__ float s_bias[kNrcBias];
  {
    const u32x4* src = (const u32x4*)Q.net;
    for (int i = threadIdx.x; i < kNrcFwdFrags * 64; i += blockDim.x) s_frag[i] = src[i];
    const float* bs = (const float*)(Q.net + kNrcFrags * 1024);
    for (int i = threadIdx.x; i < kNrcBias; i += blockDim.x) s_bias[i] = bs[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t count = MODE == 1 ? (int64_t)min((uint64_t)*Q.qcount, (uint64_t)Q.count) : Q.count;
  for (int64_t base = wave * 64; base < count; base += nwaves * 64) {
    float p[4][3], d[4][3], sg[4], beta[4];
    bool valid[4];
    bool any = false;
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
      int64_t n = base + 16 * cb + r;
      valid[cb] = n < count;
      float4 a = make_float4(0, 0, 0, 0), b = a;
      if (valid[cb]) {
        if (MODE == 0) {
          a = make_float4(Q.pos[3 * n], Q.pos[3 * n + 1], Q.pos[3 * n + 2], Q.sigma[n]);
          b = make_float4(Q.dir[3 * n], Q.dir[3 * n + 1], Q.dir[3 * n + 2], 1.0f);
        } else {
          a = Q.q[2 * n];
          b = Q.q[2 * n + 1];
        }
      }
      p[cb][0] = a.x;
      p[cb][1] = a.y;
      p[cb][2] = a.z;
      sg[cb] = a.w;
      d[cb][0] = b.x;
      d[cb][1] = b.y;
      d[cb][2] = b.z;
      beta[cb] = b.w;
      any = any || valid[cb];
    }
    if (!__any(any)) continue;
    bf16x8 X[4][3];
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
      for (int ks = 0; ks < 3; ks++)
        X[cb][ks] = feat_chunk(4 * ks + g, p[cb][0], p[cb][1], p[cb][2], d[cb][0], d[cb][1], d[cb][2], sg[cb], Q.lref);
    f32x4 acc[4][4];
    bf16x8 H[4][2];
    layer_fwd<3>(s_frag + kF0 * 64, s_bias, X, acc, lane);
    to_operand<true>(acc, H);
#pragma unroll
    for (int l = 1; l < 4; l++) {
      layer_fwd<2>(s_frag + frag_fwd(l) * 64, s_bias + 64 * l, H, acc, lane);
      to_operand<true>(acc, H);
    }
    f32x4 o[4];
    out_fwd(s_frag + kF4 * 64, s_bias + 256, H, o, lane);
    if (g == 0) {
#pragma unroll
      for (int cb = 0; cb < 4; cb++) {
        if (!valid[cb]) continue;
        int64_t n = base + 16 * cb + r;
        if (MODE == 0) {
          Q.y[3 * n] = o[cb][0];
          Q.y[3 * n + 1] = o[cb][1];
          Q.y[3 * n + 2] = o[cb][2];
        } else {
          float* px = Q.out + 3 * (size_t)Q.qpix[n];
          atomicAdd(px, beta[cb] * fmaxf(o[cb][0], 0.0f));
          atomicAdd(px + 1, beta[cb] * fmaxf(o[cb][1], 0.0f));
          atomicAdd(px + 2, beta[cb] * fmaxf(o[cb][2], 0.0f));
        }
      }
    }
  }
}

// ---------------------------------------------------------------- training
constexpr int kActStride = 72;  // bfloat16 per LDS row: 144 bytes, 16-byte aligned, rows spread over banks

struct NrcTrainArgs {
  const char* net;
  double lref;
  int32_t count;
  float norm;  // 1 / (3 count)
  const float* pos;  // records (loss mode)
  const float* dir;
  const float* sigma;
  const float* target;
  const float* feats;  // explicit features and output gradients (when non-NULL)
  const float* dy;
  float* y_out;      // nullable
  float* part;       // per-block gradients [gridDim.x][kNrcParams]
  float* loss_part;  // per-block loss sums
};

__device__ inline bf16x8 lds16(const uint16_t* buf, int row, int col) {
  return as_bf(*(const u32x4*)(buf + row * kActStride + col));
}

// Stores a B operand (units kmap(ks, g, e) of sample 16 cb + r) as rows.
__device__ inline void store_operand(uint16_t* buf, const bf16x8 (&H)[4][2], int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int cb = 0; cb < 4; cb++)
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
      u32x4 v = as_u4(H[cb][ks]);
#pragma unroll
      for (int e = 0; e < 8; e++)
        buf[kmap(ks, g, e) * kActStride + 16 * cb + r] = (uint16_t)((e & 1) ? (v[e >> 1] >> 16) : v[e >> 1]);
    }
}

// Bias gradient: sum over the 64 samples of D-layout errors (FP32).
template <int RB>
__device__ inline void bias_grad(const f32x4 (&dl)[RB][4], float* out, int nout, int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < RB; rb++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      float v = (dl[rb][0][i] + dl[rb][1][i]) + (dl[rb][2][i] + dl[rb][3][i]);
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      int u = 16 * rb + 4 * g + i;
      if (r == 0 && u < nout) out[u] = v;
    }
}

// dW[16 rb + 4 g + i][16 cbi + r] = sum over samples of delta * input, from
// the LDS rows of the errors (s_d) and of the layer input (s_in).
template <int RB, int NCB>
__device__ inline void weight_grad(const uint16_t* s_d, const uint16_t* s_in, float* out, int nout, int nin,
                                   int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < RB; rb++)
#pragma unroll
    for (int cbi = 0; cbi < NCB; cbi++) {
      f32x4 w = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 2; ks++)
        w = mfma(lds16(s_d, 16 * rb + r, 32 * ks + 8 * g), lds16(s_in, 16 * cbi + r, 32 * ks + 8 * g), w);
      int in = 16 * cbi + r;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        int o = 16 * rb + 4 * g + i;
        if (o < nout && in < nin) out[o * nin + in] = w[i];
      }
    }
}

// Errors (D layout, FP32) -> bfloat16 rows of s_d.
template <int RB>
__device__ inline void store_errors(uint16_t* s_d, const f32x4 (&dl)[RB][4], int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < RB; rb++)
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
      for (int i = 0; i < 4; i++) s_d[(16 * rb + 4 * g + i) * kActStride + 16 * cb + r] = (uint16_t)bf16_rne(dl[rb][cb][i]);
}

// ReLU derivative: keep errors of units whose (rounded) activation is positive.
__device__ inline void relu_mask(f32x4 (&acc)[4][4], const uint16_t* s_act, int lane) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < 4; rb++)
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (!bf16_positive(s_act[(16 * rb + 4 * g + i) * kActStride + 16 * cb + r])) acc[rb][cb][i] = 0.0f;
}

// One block = one wave = 64 samples: forward keeping the layer inputs,
// output errors (relative-L2 loss or given), backward, per-block gradients.
__global__ __launch_bounds__(64) void k_nrc_train(NrcTrainArgs T) {
  __shared__ u32x4 s_frag[kNrcFrags * 64];
  __shared__ float s_bias[kNrcBias];
  __shared__ uint16_t s_a0[80 * kActStride];     // features 0..79 (the input of layer 0)
  __shared__ uint16_t s_a[4][64 * kActStride];   // inputs of layers 1..4
  __shared__ uint16_t s_d[64 * kActStride];      // errors of the layer being differentiated
  {
    const u32x4* src = (const u32x4*)T.net;
    for (int i = threadIdx.x; i < kNrcFrags * 64; i += blockDim.x) s_frag[i] = src[i];
    const float* bs = (const float*)(T.net + kNrcFrags * 1024);
    for (int i = threadIdx.x; i < kNrcBias; i += blockDim.x) s_bias[i] = bs[i];
  }
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * 64;
  float* part = T.part + (size_t)blockIdx.x * kNrcParams;

  // ---- inputs
  bf16x8 X[4][3];
  bool valid[4];
#pragma unroll
  for (int cb = 0; cb < 4; cb++) {
    int64_t n = base + 16 * cb + r;
    valid[cb] = n < T.count;
#pragma unroll
    for (int ks = 0; ks < 3; ks++) {
      int c = 4 * ks + g;
      if (!valid[cb]) {
        u32x4 z = {0u, 0u, 0u, 0u};
        X[cb][ks] = as_bf(z);
      } else if (T.feats) {
        X[cb][ks] = feat_chunk_mem(T.feats + (size_t)kNrcIn * n, c);
      } else {
        X[cb][ks] = feat_chunk(c, T.pos[3 * n], T.pos[3 * n + 1], T.pos[3 * n + 2], T.dir[3 * n], T.dir[3 * n + 1],
                               T.dir[3 * n + 2], T.sigma[n], T.lref);
      }
      u32x4 v = as_u4(X[cb][ks]);
#pragma unroll
      for (int e = 0; e < 8; e++)
        if (8 * c + e < 80)
          s_a0[(8 * c + e) * kActStride + 16 * cb + r] = (uint16_t)((e & 1) ? (v[e >> 1] >> 16) : v[e >> 1]);
    }
  }
  __syncthreads();

  // ---- forward
  f32x4 acc[4][4];
  bf16x8 H[4][2];
  layer_fwd<3>(s_frag + kF0 * 64, s_bias, X, acc, lane);
  to_operand<true>(acc, H);
  store_operand(s_a[0], H, lane);
#pragma unroll
  for (int l = 1; l < 4; l++) {
    layer_fwd<2>(s_frag + frag_fwd(l) * 64, s_bias + 64 * l, H, acc, lane);
    to_operand<true>(acc, H);
    store_operand(s_a[l], H, lane);
  }
  f32x4 o[4];
  out_fwd(s_frag + kF4 * 64, s_bias + 256, H, o, lane);

  // ---- output errors
  f32x4 d4[1][4];
  float lsum = 0.0f;
#pragma unroll
  for (int cb = 0; cb < 4; cb++) {
    d4[0][cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int64_t n = base + 16 * cb + r;
    if (g == 0 && valid[cb]) {
#pragma unroll
      for (int i = 0; i < 3; i++) {
        float yv = o[cb][i];
        if (T.y_out) T.y_out[3 * n + i] = yv;
        float dyv;
        if (T.dy) {
          dyv = T.dy[3 * n + i];
        } else {
          float den = yv * yv + 0.01f;
          float e = yv - T.target[3 * n + i];
          lsum = lsum + e * e / den;
          dyv = 2.0f * e / den * T.norm;
        }
        d4[0][cb][i] = dyv;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if (lane == 0) T.loss_part[blockIdx.x] = lsum;
  bias_grad<1>(d4, part + nrc_off_b(4), 3, lane);
  store_errors<1>(s_d, d4, lane);
  __syncthreads();
  weight_grad<1, 4>(s_d, s_a[3], part + nrc_off_w(4), 3, 64, lane);

  // ---- delta3 = W4^T delta4, masked
  bf16x8 Bd[4][2];
  {
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int cb = 0; cb < 4; cb++) Bd[cb][0] = dpack<false>(d4[0][cb], z);
#pragma unroll
    for (int rb = 0; rb < 4; rb++) {
      bf16x8 a = as_bf(s_frag[(kB4 + rb) * 64 + lane]);
#pragma unroll
      for (int cb = 0; cb < 4; cb++) acc[rb][cb] = mfma(a, Bd[cb][0], z);
    }
  }
  relu_mask(acc, s_a[3], lane);
  // ---- layers 3, 2, 1: gradients, then the errors one layer down
#pragma unroll
  for (int l = 3; l >= 1; l--) {
    bias_grad<4>(acc, part + nrc_off_b(l), 64, lane);
    __syncthreads();  // s_d's previous errors are consumed
    store_errors<4>(s_d, acc, lane);
    __syncthreads();
    weight_grad<4, 4>(s_d, s_a[l - 1], part + nrc_off_w(l), 64, 64, lane);
    to_operand<false>(acc, Bd);
    const int fb = frag_bwd(l);
#pragma unroll
    for (int rb = 0; rb < 4; rb++)
#pragma unroll
      for (int cb = 0; cb < 4; cb++) acc[rb][cb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
      for (int rb = 0; rb < 4; rb++) {
        bf16x8 a = as_bf(s_frag[(fb + rb * 2 + ks) * 64 + lane]);
#pragma unroll
        for (int cb = 0; cb < 4; cb++) acc[rb][cb] = mfma(a, Bd[cb][ks], acc[rb][cb]);
      }
    relu_mask(acc, s_a[l - 1], lane);
  }
  // ---- layer 0
  bias_grad<4>(acc, part + nrc_off_b(0), 64, lane);
  __syncthreads();
  store_errors<4>(s_d, acc, lane);
  __syncthreads();
  weight_grad<4, 5>(s_d, s_a0, part + nrc_off_w(0), 64, kNrcIn, lane);
}

struct NrcReduceArgs {
  const float* part;
  int32_t nblk;
  float* grads;  // nullable: the summed gradient
  int32_t adam;
  float* master;
  float* m;
  float* v;
  float lr, beta1, beta2, eps, c1, c2;  // c = 1 - beta^step
  const float* loss_part;
  float* loss;  // nullable: sum of loss_part times norm
  float norm;
  float* ema;    // nullable: weight average, updated after the Adam step
  float* infer;  // its bias-corrected value
  float ema_b, ema_c;  // e, 1 - e^step
};

// Gradient = sum of the blocks' parts in block order (deterministic); then
// the Adam update of the FP32 master weights.
__global__ void k_nrc_reduce(NrcReduceArgs A) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNrcParams) {
    float s = 0.0f;
    for (int b = 0; b < A.nblk; b++) s += A.part[(size_t)b * kNrcParams + p];
    if (A.grads) A.grads[p] = s;
    if (A.adam) {
      float mm = A.beta1 * A.m[p] + (1.0f - A.beta1) * s;
      float vv = A.beta2 * A.v[p] + (1.0f - A.beta2) * s * s;
      A.m[p] = mm;
      A.v[p] = vv;
      float mh = mm / A.c1, vh = vv / A.c2;
      float w = A.master[p] - A.lr * mh / (sqrtf(vh) + A.eps);
      A.master[p] = w;
      if (A.ema) {
        float e = A.ema_b * A.ema[p] + (1.0f - A.ema_b) * w;
        A.ema[p] = e;
        A.infer[p] = e / A.ema_c;
      }
    }
  }
  if (p == 0 && A.loss) {
    float l = 0.0f;
    for (int b = 0; b < A.nblk; b++) l += A.loss_part[b];
    *A.loss = l * A.norm;
  }
}

// ---------------------------------------------------------------- training records
// Records per path: vertices k < min(count, kv) with a positive throughput.
__global__ void k_nrc_count(const float4* __restrict__ vrec, const float4* __restrict__ path_l, int32_t n, int32_t kv,
                            uint32_t* __restrict__ cnt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t nv = min(__float_as_uint(path_l[j].w), (uint32_t)kv), c = 0;
  for (uint32_t k = 0; k < nv; k++) c += vrec[((size_t)j * kv + k) * 3 + 1].w > 0.0f ? 1u : 0u;
  cnt[j] = c;
}

// Exclusive prefix sum of n counts in one block of 1024 threads (each
// thread a consecutive run); off[n] = total.
__global__ __launch_bounds__(1024) void k_nrc_scan(const uint32_t* __restrict__ cnt, int32_t n,
                                                   uint32_t* __restrict__ off) {
  __shared__ uint32_t s[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  uint32_t sum = 0;
  for (int i = lo; i < hi; i++) sum += cnt[i];
  s[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    uint32_t v = t >= d ? s[t - d] : 0u;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  uint32_t run = s[t] - sum;
  for (int i = lo; i < hi; i++) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[n] = s[1023];
}

struct NrcEmitArgs {
  const float4* vrec;
  const float4* path_l;
  const uint32_t* off;
  int32_t n, kv;
  int64_t capacity;
  float* pos;
  float* dir;
  float* sigma;
  float* target;
  int32_t* tag;  // nullable
};

// Compacted records in (path, vertex) order: target = (L_final - L_before) / beta.
__global__ void k_nrc_emit(NrcEmitArgs E) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= E.n) return;
  float4 lf = E.path_l[j];
  uint32_t nv = min(__float_as_uint(lf.w), (uint32_t)E.kv);
  int64_t c = E.off[j];
  for (uint32_t k = 0; k < nv; k++) {
    const float4* q = E.vrec + ((size_t)j * E.kv + k) * 3;
    float4 a = q[0], b = q[1], lb = q[2];
    if (!(b.w > 0.0f)) continue;
    if (c < E.capacity) {
      E.pos[3 * c] = a.x;
      E.pos[3 * c + 1] = a.y;
      E.pos[3 * c + 2] = a.z;
      E.dir[3 * c] = b.x;
      E.dir[3 * c + 1] = b.y;
      E.dir[3 * c + 2] = b.z;
      E.sigma[c] = a.w;
      E.target[3 * c] = (lf.x - lb.x) / b.w;
      E.target[3 * c + 1] = (lf.y - lb.y) / b.w;
      E.target[3 * c + 2] = (lf.z - lb.z) / b.w;
      if (E.tag) E.tag[c] = 16 * j + (int32_t)k;
    }
    c++;
  }
}

// Largest extinction of a grid: wave and block maxima, then one atomic per
// block, skipped when it cannot raise the running maximum (a single address
// taking one atomic per wave would serialise).
__device__ inline void block_max_to(uint32_t v, uint32_t* out) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
  __shared__ uint32_t s_max[16];
  if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = s_max[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); k++) m = max(m, s_max[k]);
    if (m > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(out, m);
  }
}
__global__ void k_max_sigma32(const TetRec32* __restrict__ rec, int64_t n, uint32_t* out) {
  uint32_t v = 0u;  // extinction >= 0: its bits order like the values
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = max(v, rec[i].w[3]);
  block_max_to(v, out);
}
__global__ void k_max_sigma48(const TetRec* __restrict__ rec, int64_t n, uint32_t* out) {
  uint32_t v = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = max(v, __float_as_uint(rec[i].sigma));
  block_max_to(v, out);
}

__global__ void k_zero_word(uint32_t* p) { *p = 0u; }

// ---------------------------------------------------------------- host
namespace {

struct Scratch {
  void* p = nullptr;
  explicit Scratch(size_t bytes) : p(dev_alloc(bytes)) {}
  ~Scratch() { dev_free(p); }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  char* c() const { return (char*)p; }
};

int check_nrc(const tet_nrc* nrc) {
  if (!nrc || !nrc->master || !nrc->net) return fail(TET_ERR_INVALID_ARG, "radiance cache is NULL");
  return TET_OK;
}

// Packs the master weights (training) and, with a weight average, the
// weights the queries use.
int pack(tet_nrc* nrc, hipStream_t st) {
  int total = kNrcFrags * 256 + kNrcBias;
  hipLaunchKernelGGL(k_nrc_pack, dim3((total + 255) / 256), dim3(256), 0, st, nrc->master, nrc->net);
  if (nrc->opts.ema > 0.0f)
    hipLaunchKernelGGL(k_nrc_pack, dim3((total + 255) / 256), dim3(256), 0, st, nrc->infer, nrc->net_infer);
  TV_HIP(hipGetLastError());
  return TET_OK;
}

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator.
uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One forward/backward launch over `count` samples; partial gradients and
// loss sums per block of 64.
int launch_train(const tet_nrc* nrc, int32_t count, const float* pos, const float* dir, const float* sigma,
                 const float* target, const float* feats, const float* dy, float* y_out, float* part, float* loss_part,
                 hipStream_t st) {
  NrcTrainArgs T;
  memset(&T, 0, sizeof(T));
  T.net = nrc->net;
  T.lref = nrc->opts.sigma_ref > 0.0f ? std::log1p((double)nrc->opts.sigma_ref) : 1.0;
  T.count = count;
  T.norm = (float)(1.0 / (3.0 * (double)count));
  T.pos = pos;
  T.dir = dir;
  T.sigma = sigma;
  T.target = target;
  T.feats = feats;
  T.dy = dy;
  T.y_out = y_out;
  T.part = part;
  T.loss_part = loss_part;
  int nblk = (count + 63) / 64;
  hipLaunchKernelGGL(k_nrc_train, dim3(nblk), dim3(64), 0, st, T);
  TV_HIP(hipGetLastError());
  return TET_OK;
}

int launch_reduce(tet_nrc* nrc, int32_t count, const float* part, const float* loss_part, float* grads, float* loss,
                  bool adam, hipStream_t st) {
  NrcReduceArgs A;
  memset(&A, 0, sizeof(A));
  A.part = part;
  A.nblk = (count + 63) / 64;
  A.grads = grads;
  A.loss_part = loss_part;
  A.loss = loss;
  A.norm = (float)(1.0 / (3.0 * (double)count));
  if (adam) {
    nrc->step++;
    const tet_nrc_opts& o = nrc->opts;
    A.adam = 1;
    A.master = nrc->master;
    A.m = nrc->m;
    A.v = nrc->v;
    A.lr = o.lr;
    A.beta1 = o.beta1;
    A.beta2 = o.beta2;
    A.eps = o.eps;
    A.c1 = (float)(1.0 - std::pow((double)o.beta1, (double)nrc->step));
    A.c2 = (float)(1.0 - std::pow((double)o.beta2, (double)nrc->step));
    if (o.ema > 0.0f) {
      A.ema = nrc->ema;
      A.infer = nrc->infer;
      A.ema_b = o.ema;
      A.ema_c = (float)(1.0 - std::pow((double)o.ema, (double)nrc->step));
    }
  }
  hipLaunchKernelGGL(k_nrc_reduce, dim3((kNrcParams + 255) / 256), dim3(256), 0, st, A);
  TV_HIP(hipGetLastError());
  if (adam) return pack(nrc, st);
  return TET_OK;
}

// `steps` Adam steps over `count` device-resident records split in equal
// consecutive batches; the batch losses (before each step) go to loss_dev
// (device, `steps` floats); *used = the steps taken.
int train_records(tet_nrc* nrc, int64_t count, const float* pos, const float* dir, const float* sigma,
                  const float* target, int steps, float* loss_dev, int* used, hipStream_t st) {
  *used = 0;
  if (count <= 0) return TET_OK;
  int64_t per = (count + steps - 1) / steps;
  int nblk = (int)((per + 63) / 64);
  Scratch part((size_t)nblk * kNrcParams * 4 + (size_t)nblk * 4);
  if (!part.p) return fail(TET_ERR_OUT_OF_MEMORY, "radiance cache: gradient scratch");
  float* pp = (float*)part.c();
  float* lp = pp + (size_t)nblk * kNrcParams;
  for (int k = 0; k < steps; k++) {
    int64_t a = (int64_t)k * per, b = std::min<int64_t>(count, a + per);
    if (b <= a) break;
    int32_t c = (int32_t)(b - a);
    if (int rc = launch_train(nrc, c, pos + 3 * a, dir + 3 * a, sigma + a, target + 3 * a, nullptr, nullptr, nullptr,
                              pp, lp, st))
      return rc;
    if (int rc = launch_reduce(nrc, c, pp, lp, nullptr, loss_dev + k, true, st)) return rc;
    (*used)++;
  }
  TV_HIP(hipStreamSynchronize(st));  // the gradient scratch is released on return
  return TET_OK;
}

int resolve_sigma_ref(tet_nrc* nrc, const tet_grid* g, hipStream_t st) {
  if (nrc->opts.sigma_ref > 0.0f) return TET_OK;
  Scratch s(4);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "radiance cache: scratch");
  uint32_t* d = (uint32_t*)s.c();
  hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, st, d);
  int64_t n = g->n;
  unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  if (g->rec32) hipLaunchKernelGGL(k_max_sigma32, dim3(blocks), dim3(256), 0, st, g->rec32, n, d);
  else hipLaunchKernelGGL(k_max_sigma48, dim3(blocks), dim3(256), 0, st, g->rec, n, d);
  TV_HIP(hipGetLastError());
  uint32_t h = 0;
  TV_HIP(hipMemcpyAsync(&h, d, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  float v;
  memcpy(&v, &h, 4);
  nrc->opts.sigma_ref = v > 0.0f ? v : 1.0f;
  return TET_OK;
}

}  // namespace

int nrc_resolve_sigma_ref(tet_nrc* n, const tet_grid* g, hipStream_t st) { return resolve_sigma_ref(n, g, st); }

int nrc_create(const tet_nrc_opts* in, tet_nrc** out) {
  if (!out) return fail(TET_ERR_INVALID_ARG, "tet_nrc_create: out is NULL");
  *out = nullptr;
  tet_nrc_opts o;
  if (in) o = *in;
  else tet_nrc_opts_defaults(&o);
  if (o.truncate_bounce < 1 || o.train_paths < 1 || o.train_paths > (1 << 24) || o.train_vertices < 1 ||
      o.train_vertices > 16 || o.train_steps < 1 || !(o.lr > 0.0f) || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) ||
      !(o.beta2 >= 0.0f && o.beta2 < 1.0f) || !(o.eps > 0.0f) || !(o.sigma_ref >= 0.0f) ||
      !(o.ema >= 0.0f && o.ema < 1.0f))
    return fail(TET_ERR_INVALID_ARG, "tet_nrc_create: bad options");
  tet_nrc* n = new tet_nrc();
  memset(n, 0, sizeof(*n));
  n->opts = o;
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return fail(TET_ERR_DEVICE, "tet_nrc_create: no device");
  }
  size_t pb = (size_t)kNrcParams * 4;
  if (hipMalloc(&n->master, pb) != hipSuccess || hipMalloc(&n->m, pb) != hipSuccess ||
      hipMalloc(&n->v, pb) != hipSuccess || hipMalloc(&n->net, kNrcNetBytes) != hipSuccess ||
      hipMalloc(&n->ema, pb) != hipSuccess || hipMalloc(&n->infer, pb) != hipSuccess ||
      hipMalloc(&n->net_infer, kNrcNetBytes) != hipSuccess) {
    (void)hipGetLastError();
    nrc_free(n);
    return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_create: device memory");
  }
  // He-uniform weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)), zero biases
  std::vector<float> P(kNrcParams, 0.0f);
  uint64_t x = o.seed;
  for (int l = 0; l < 5; l++) {
    int fi = l == 0 ? kNrcIn : 64, fo = l == 4 ? 3 : 64;
    double a = std::sqrt(6.0 / fi);
    for (int k = 0; k < fo * fi; k++) {
      double u = (double)(splitmix64(x) >> 11) * 0x1p-53;
      P[nrc_off_w(l) + k] = (float)((2.0 * u - 1.0) * a);
    }
  }
  int rc = nrc_import(n, P.data(), 0, nullptr);
  if (rc) {
    nrc_free(n);
    return rc;
  }
  *out = n;
  return TET_OK;
}

void nrc_free(tet_nrc* n) {
  if (!n) return;
  if (n->master) (void)hipFree(n->master);
  if (n->m) (void)hipFree(n->m);
  if (n->v) (void)hipFree(n->v);
  if (n->net) (void)hipFree(n->net);
  if (n->ema) (void)hipFree(n->ema);
  if (n->infer) (void)hipFree(n->infer);
  if (n->net_infer) (void)hipFree(n->net_infer);
  delete n;
}

int nrc_export(const tet_nrc* n, float* params, int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (!params) return fail(TET_ERR_INVALID_ARG, "tet_nrc_export: params is NULL");
  TV_HIP(hipMemcpyAsync(params, n->master, (size_t)kNrcParams * 4,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_import(tet_nrc* n, const float* params, int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (!params) return fail(TET_ERR_INVALID_ARG, "tet_nrc_import: params is NULL");
  size_t pb = (size_t)kNrcParams * 4;
  TV_HIP(hipMemcpyAsync(n->master, params, pb, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  std::vector<float> z(kNrcParams, 0.0f);
  TV_HIP(hipMemcpyAsync(n->m, z.data(), pb, hipMemcpyHostToDevice, st));
  TV_HIP(hipMemcpyAsync(n->v, z.data(), pb, hipMemcpyHostToDevice, st));
  TV_HIP(hipMemcpyAsync(n->ema, z.data(), pb, hipMemcpyHostToDevice, st));
  TV_HIP(hipMemcpyAsync(n->infer, n->master, pb, hipMemcpyDeviceToDevice, st));
  n->step = 0;
  if (int rc = pack(n, st)) return rc;
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_export_inference(const tet_nrc* n, float* params, int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (!params) return fail(TET_ERR_INVALID_ARG, "tet_nrc_export_inference: params is NULL");
  TV_HIP(hipMemcpyAsync(params, n->opts.ema > 0.0f ? n->infer : n->master, (size_t)kNrcParams * 4,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_infer(const tet_nrc* n, int64_t count, const float* pos, const float* dir, const float* sigma, float* y,
              int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (count < 0 || (count && (!pos || !dir || !sigma || !y))) return fail(TET_ERR_INVALID_ARG, "tet_nrc_infer: bad arguments");
  if (!(n->opts.sigma_ref > 0.0f)) return fail(TET_ERR_INVALID_ARG, "tet_nrc_infer: sigma_ref is not set");
  if (count == 0) return TET_OK;
  size_t b3 = (size_t)count * 12, b1 = (size_t)count * 4;
  Scratch s(on_device ? 16 : 3 * b3 + b1);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_infer: scratch");
  NrcQueryArgs Q;
  memset(&Q, 0, sizeof(Q));
  Q.net = n->query_net();
  Q.lref = std::log1p((double)n->opts.sigma_ref);
  Q.count = count;
  if (on_device) {
    Q.pos = pos;
    Q.dir = dir;
    Q.sigma = sigma;
    Q.y = y;
  } else {
    float* dp = (float*)s.c();
    Q.pos = dp;
    Q.dir = dp + 3 * count;
    Q.y = dp + 6 * count;
    Q.sigma = dp + 9 * count;
    TV_HIP(hipMemcpyAsync((void*)Q.pos, pos, b3, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)Q.dir, dir, b3, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)Q.sigma, sigma, b1, hipMemcpyHostToDevice, st));
  }
  int64_t waves = (count + 63) / 64;
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 2048));
  hipLaunchKernelGGL(k_nrc_query<0>, dim3(grid), dim3(256), 0, st, Q);
  TV_HIP(hipGetLastError());
  if (!on_device) TV_HIP(hipMemcpyAsync(y, Q.y, b3, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_query_pass(const tet_nrc* n, const float4* q, const uint32_t* qpix, const uint32_t* qcount, float* out,
                   int64_t capacity, hipStream_t st) {
  if (capacity <= 0) return TET_OK;
  NrcQueryArgs Q;
  memset(&Q, 0, sizeof(Q));
  Q.net = n->query_net();
  Q.lref = std::log1p((double)n->opts.sigma_ref);
  Q.count = capacity;
  Q.q = q;
  Q.qpix = qpix;
  Q.qcount = qcount;
  Q.out = out;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // persistent blocks (the number of queries is on the device): 4 per CU,
  // as many as the weights' 40 KB of LDS per block allow
  int64_t waves = (capacity + 63) / 64;
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, (int64_t)cus * 4));
  hipLaunchKernelGGL(k_nrc_query<1>, dim3(grid), dim3(256), 0, st, Q);
  TV_HIP(hipGetLastError());
  return TET_OK;
}

int nrc_forward_backward(const tet_nrc* n, int32_t count, const float* feats, const float* dy, float* y, float* grads,
                         int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (count < 1 || count > (1 << 20) || !feats || !dy || !grads)
    return fail(TET_ERR_INVALID_ARG, "tet_nrc_forward_backward: bad arguments");
  int nblk = (count + 63) / 64;
  size_t bf = (size_t)count * kNrcIn * 4, b3 = (size_t)count * 12, bg = (size_t)kNrcParams * 4;
  size_t part_b = (size_t)nblk * kNrcParams * 4 + (size_t)nblk * 4;
  Scratch s(part_b + (on_device ? 0 : bf + 2 * b3 + bg) + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_forward_backward: scratch");
  float* pp = (float*)s.c();
  float* lp = pp + (size_t)nblk * kNrcParams;
  const float *df = feats, *ddy = dy;
  float *dyo = y, *dg = grads;
  if (!on_device) {
    char* h = s.c() + ((part_b + 255) & ~(size_t)255);
    df = (const float*)h;
    ddy = (const float*)(h + bf);
    dyo = y ? (float*)(h + bf + b3) : nullptr;
    dg = (float*)(h + bf + 2 * b3);
    TV_HIP(hipMemcpyAsync((void*)df, feats, bf, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)ddy, dy, b3, hipMemcpyHostToDevice, st));
  }
  if (int rc = launch_train(n, count, nullptr, nullptr, nullptr, nullptr, df, ddy, dyo, pp, lp, st)) return rc;
  if (int rc = launch_reduce(const_cast<tet_nrc*>(n), count, pp, lp, dg, nullptr, false, st)) return rc;
  if (!on_device) {
    TV_HIP(hipMemcpyAsync(grads, dg, bg, hipMemcpyDeviceToHost, st));
    if (y) TV_HIP(hipMemcpyAsync(y, dyo, b3, hipMemcpyDeviceToHost, st));
  }
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_train_batch(tet_nrc* n, int32_t count, const float* pos, const float* dir, const float* sigma,
                    const float* target, float* loss, int32_t on_device, hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (count < 1 || count > (1 << 20) || !pos || !dir || !sigma || !target)
    return fail(TET_ERR_INVALID_ARG, "tet_nrc_train_batch: bad arguments");
  if (!(n->opts.sigma_ref > 0.0f)) return fail(TET_ERR_INVALID_ARG, "tet_nrc_train_batch: sigma_ref is not set");
  size_t b3 = (size_t)count * 12, b1 = (size_t)count * 4;
  Scratch s(on_device ? 256 : 3 * b3 + b1 + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_train_batch: scratch");
  const float *dp = pos, *dd = dir, *ds = sigma, *dt = target;
  float* dl = (float*)s.c();
  if (!on_device) {
    float* h = (float*)(s.c() + 256);
    dp = h;
    dd = h + 3 * (size_t)count;
    dt = h + 6 * (size_t)count;
    ds = h + 9 * (size_t)count;
    TV_HIP(hipMemcpyAsync((void*)dp, pos, b3, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)dd, dir, b3, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)dt, target, b3, hipMemcpyHostToDevice, st));
    TV_HIP(hipMemcpyAsync((void*)ds, sigma, b1, hipMemcpyHostToDevice, st));
  }
  int used = 0;
  if (int rc = train_records(n, count, dp, dd, ds, dt, 1, dl, &used, st)) return rc;
  if (loss) {
    TV_HIP(hipMemcpyAsync(loss, dl, 4, hipMemcpyDeviceToHost, st));
    TV_HIP(hipStreamSynchronize(st));
  }
  return TET_OK;
}

namespace {
// Compacts traced training paths (up to kv vertex records each) into record
// arrays (pos 3, dir 3, sigma 1, target 3 floats, tag) of capacity `cap`;
// *count = the number of records.
int compact_records(int32_t np, int32_t kv, const float4* vrec, const float4* pl, float* pos, float* dir,
                    float* sigma, float* target, int32_t* tag, int64_t cap, int64_t* count, hipStream_t st) {
  size_t cb = ((size_t)np + 1) * 4;
  Scratch s(2 * cb + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "radiance cache: compaction scratch");
  uint32_t* cnt = (uint32_t*)s.c();
  uint32_t* off = (uint32_t*)(s.c() + cb + 128);
  hipLaunchKernelGGL(k_nrc_count, dim3((np + 255) / 256), dim3(256), 0, st, vrec, pl, np, kv, cnt);
  hipLaunchKernelGGL(k_nrc_scan, dim3(1), dim3(1024), 0, st, cnt, np, off);
  NrcEmitArgs E{vrec, pl, off, np, kv, cap, pos, dir, sigma, target, tag};
  hipLaunchKernelGGL(k_nrc_emit, dim3((np + 255) / 256), dim3(256), 0, st, E);
  TV_HIP(hipGetLastError());
  uint32_t total = 0;
  TV_HIP(hipMemcpyAsync(&total, off + np, 4, hipMemcpyDeviceToHost, st));
  TV_HIP(hipStreamSynchronize(st));
  *count = total;
  return TET_OK;
}

// Traces the frame's training paths and compacts their records.
int collect_device(const tet_nrc* n, const tet_grid* g, const tet_camera* cam, const tet_medium* med,
                   const tet_light* light, uint64_t frame_seed, const tet_render_opts* ro, float* pos, float* dir,
                   float* sigma, float* target, int32_t* tag, int64_t cap, int64_t* count, hipStream_t st,
                   float* trace_ms) {
  const int32_t np = n->opts.train_paths, kv = n->opts.train_vertices;
  size_t vb = (size_t)np * kv * 48, lb = (size_t)np * 16;
  Scratch s(vb + lb + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "radiance cache: training-path scratch");
  float4* vrec = (float4*)s.c();
  float4* pl = (float4*)(s.c() + vb);
  if (int rc = trace_training_paths(g, cam, med, light, frame_seed, ro, np, kv, vrec, pl, st, trace_ms)) return rc;
  return compact_records(np, kv, vrec, pl, pos, dir, sigma, target, tag, cap, count, st);
}
}  // namespace

// Compaction and train_steps Adam steps over training paths a render traced
// (vertex records and path radiance on the device).
int nrc_train_paths(tet_nrc* n, const float4* vrec, const float4* pl, int32_t np, int32_t kv, hipStream_t st,
                    int64_t* records, double* loss) {
  int64_t cap = (int64_t)np * kv;
  int steps = n->opts.train_steps;
  Scratch s(40 * (size_t)cap + (size_t)steps * 4 + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "radiance cache: record scratch");
  float* h = (float*)s.c();
  float *dp = h, *dd = h + 3 * cap, *dt = h + 6 * cap, *ds = h + 9 * cap, *dl = h + 10 * cap;
  int64_t c = 0;
  if (int rc = compact_records(np, kv, vrec, pl, dp, dd, ds, dt, nullptr, cap, &c, st)) return rc;
  int used = 0;
  if (int rc = train_records(n, c, dp, dd, ds, dt, steps, dl, &used, st)) return rc;
  if (records) *records = c;
  if (loss) {
    std::vector<float> hl(std::max(used, 1), 0.0f);
    if (used) TV_HIP(hipMemcpy(hl.data(), dl, (size_t)used * 4, hipMemcpyDeviceToHost));
    double sum = 0.0;
    for (int k = 0; k < used; k++) sum += hl[k];
    *loss = used ? sum / used : 0.0;
  }
  return TET_OK;
}

int nrc_collect(const tet_nrc* n, const tet_grid* g, const tet_camera* cam, const tet_medium* med,
                const tet_light* light, uint64_t frame_seed, const tet_render_opts* ro, float* pos, float* dir,
                float* sigma, float* target, int32_t* tag, int64_t capacity, int64_t* count, int32_t on_device,
                hipStream_t st) {
  if (int rc = check_nrc(n)) return rc;
  if (!g || !pos || !dir || !sigma || !target || !count || capacity < 0)
    return fail(TET_ERR_INVALID_ARG, "tet_nrc_collect: bad arguments");
  *count = 0;
  int64_t cap = (int64_t)n->opts.train_paths * n->opts.train_vertices;
  size_t b3 = (size_t)cap * 12, b1 = (size_t)cap * 4;
  Scratch s(3 * b3 + 2 * b1 + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_collect: scratch");
  float* h = (float*)s.c();
  float *dp = h, *dd = h + 3 * cap, *dt = h + 6 * cap, *ds = h + 9 * cap;
  int32_t* dg = (int32_t*)(h + 10 * cap);
  int64_t c = 0;
  float tms = 0.0f;
  if (int rc = collect_device(n, g, cam, med, light, frame_seed, ro, dp, dd, ds, dt, dg, cap, &c, st, &tms)) return rc;
  *count = c;
  if (c > capacity) return fail(TET_ERR_CAPACITY, "tet_nrc_collect: more records than capacity");
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (c) {
    TV_HIP(hipMemcpyAsync(pos, dp, (size_t)c * 12, k, st));
    TV_HIP(hipMemcpyAsync(dir, dd, (size_t)c * 12, k, st));
    TV_HIP(hipMemcpyAsync(target, dt, (size_t)c * 12, k, st));
    TV_HIP(hipMemcpyAsync(sigma, ds, (size_t)c * 4, k, st));
    if (tag) TV_HIP(hipMemcpyAsync(tag, dg, (size_t)c * 4, k, st));
  }
  TV_HIP(hipStreamSynchronize(st));
  return TET_OK;
}

int nrc_train_frame(tet_nrc* n, const tet_grid* g, const tet_camera* cam, const tet_medium* med,
                    const tet_light* light, uint64_t frame_seed, const tet_render_opts* ro, hipStream_t st,
                    tet_nrc_stats* stats) {
  if (int rc = check_nrc(n)) return rc;
  if (!g) return fail(TET_ERR_INVALID_ARG, "tet_nrc_train_frame: grid is NULL");
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
  TV_HIP(hipEventRecord(e0, st));
  if (int rc = resolve_sigma_ref(n, g, st)) return rc;
  const int32_t np = n->opts.train_paths, kv = n->opts.train_vertices;
  size_t vb = (size_t)np * kv * 48, lb = (size_t)np * 16;
  Scratch s(vb + lb + 256);
  if (!s.p) return fail(TET_ERR_OUT_OF_MEMORY, "tet_nrc_train_frame: scratch");
  float4* vrec = (float4*)s.c();
  float4* pl = (float4*)(s.c() + vb);
  float tms = 0.0f;
  if (int rc = trace_training_paths(g, cam, med, light, frame_seed, ro, np, kv, vrec, pl, st, &tms)) return rc;
  int64_t c = 0;
  double loss = 0.0;
  if (int rc = nrc_train_paths(n, vrec, pl, np, kv, st, &c, &loss)) return rc;
  TV_HIP(hipEventRecord(e1, st));
  TV_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  TV_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (stats) {
    stats->records = c;
    stats->loss = loss;
    stats->ms = ms;
    stats->trace_ms = tms;
  }
  return TET_OK;
}

}  // namespace tv
