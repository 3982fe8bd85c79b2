// common.h -- shared definitions of libtetvol (device helpers, grid object,
// error state, device-memory cache).  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "tetvol.h"

namespace tv {

// Lattice: world coordinates times 2^20 are exact integers.
constexpr int kLatBits = 20;
constexpr int32_t kLatS = 1 << kLatBits;
constexpr uint32_t kBoundary = 0xFFFFFFFFu;
constexpr uint64_t kEmptyKey = ~0ull;  // never a packed vertex (coords <= 2^20 < 2^21 - 1)
constexpr int kMaxLevels = 13;          // pyramid levels for n <= 4096

// Traversal record of one tet: everything a walk step reads, 48 bytes,
// fetched as three 16-byte loads.
struct alignas(16) TetRec {
  float off[4];      // face plane offsets n_f . v in world units
  uint32_t nbr[4];   // (index << 2) | back face, or kBoundary
  uint32_t codes;    // byte f: orientation code 2 N + s of face f (outward normal = (-1)^s dir_N)
  float sigma;       // extinction
  float majorant;    // >= sigma
  uint32_t pad;
};
static_assert(sizeof(TetRec) == 48, "record size");

// Compact traversal record, 32 bytes (two 16-byte loads, never straddling a
// 64-byte sector); the same values as TetRec for grids of < 2^27 tets with
// tight majorants:
//   w[0..2]: the 4 plane offsets n_f . v in lattice units as 23-bit two's
//            complement integers, packed little-endian at bits 0, 23, 46, 69
//            (world offset = offset * 2^-20, exact in FP32);
//   w[3]:    extinction (FP32 bits);
//   w[4+f]:  neighbour index across face f (27 bits; kLink27Boundary on the
//            boundary) | face f's orientation code 2 N + s as N << 27 and
//            s << 31 (the sign then flips a float with one masked XOR).
struct alignas(32) TetRec32 {
  uint32_t w[8];
};
static_assert(sizeof(TetRec32) == 32, "compact record size");
constexpr uint32_t kLink27Boundary = (1u << 27) - 1;
__host__ __device__ inline uint32_t code_bits32(uint32_t code) { return ((code >> 1) << 27) | ((code & 1u) << 31); }
__host__ __device__ inline uint32_t code_of32(uint32_t w) { return (((w >> 27) & 15u) << 1) | (w >> 31); }
constexpr int64_t kMaxTets32 = (1ll << 27) - 1;

// The 9 plane directions of these grids' faces; a face's outward normal is
// +dir_N or -dir_N, its orientation code 2 N + (0 or 1).
//   0 (1,0,0)  1 (0,1,0)  2 (0,0,1)  3 (1,1,0)  4 (1,-1,0)
//   5 (1,0,1)  6 (1,0,-1) 7 (0,1,1)  8 (0,1,-1)
__host__ __device__ inline int dir_code(const int un[3]) {
  int s = 0, v[3] = {un[0], un[1], un[2]};
  int first = v[0] != 0 ? v[0] : (v[1] != 0 ? v[1] : v[2]);
  if (first < 0) {
    s = 1;
    v[0] = -v[0];
    v[1] = -v[1];
    v[2] = -v[2];
  }
  int N = -1;
  if (v[0] == 1 && v[1] == 0 && v[2] == 0) N = 0;
  else if (v[0] == 0 && v[1] == 1 && v[2] == 0) N = 1;
  else if (v[0] == 0 && v[1] == 0 && v[2] == 1) N = 2;
  else if (v[0] == 1 && v[1] == 1 && v[2] == 0) N = 3;
  else if (v[0] == 1 && v[1] == -1 && v[2] == 0) N = 4;
  else if (v[0] == 1 && v[1] == 0 && v[2] == 1) N = 5;
  else if (v[0] == 1 && v[1] == 0 && v[2] == -1) N = 6;
  else if (v[0] == 0 && v[1] == 1 && v[2] == 1) N = 7;
  else if (v[0] == 0 && v[1] == 1 && v[2] == -1) N = 8;
  return N < 0 ? -1 : 2 * N + s;
}

// Density pyramid: level 0 is the input volume; levels 1..L hold per cell
// min, max (FP32) and the FP64 sum of its 8 children combined as
// ((c000 + c100) + (c010 + c110)) + ((c001 + c101) + (c011 + c111)).
struct Pyramid {
  const float* dens;
  int32_t n, L;
  const float* mn[kMaxLevels];
  const float* mx[kMaxLevels];
  const double* sum[kMaxLevels];
  // sparse volume (zero outside 8^3 bricks; dens and levels 1, 2 unused):
  // brick index at each brick position (nb^3, -1 = empty), and per brick
  // its 512 voxels (bval) and its level-1 (64 cells) and level-2 (8 cells)
  // statistics; levels >= 3 are dense as above
  const int32_t* bmap;
  int32_t nb;
  const float* bval;
  const float* bmn[3];
  const float* bmx[3];
  const double* bsum[3];
};
constexpr int kBrickBits = 3;  // sparse bricks of 8^3 voxels

// Camera quantities of the camera criterion, FP64.
struct CamCrit {
  double pos[3], f[3], side[4][3];
  double kpx2, tgt2;
};

// Camera ray frame, FP32 (rounded once from FP64).
struct Frame {
  float pos[3], f[3], r[3], u[3];
  float tan_x, tan_y;
  int32_t w, h;
};

struct WantParams {
  int32_t mode, uniform_depth, max_depth, pad;
  double tau;
  uint64_t rand_seed;
  int32_t rand_thresh;
};

// ---------------------------------------------------------------- device helpers
__host__ __device__ inline uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

__host__ __device__ inline uint64_t pack_vertex(int32_t x, int32_t y, int32_t z) {
  return (uint64_t)(uint32_t)x | ((uint64_t)(uint32_t)y << 21) | ((uint64_t)(uint32_t)z << 42);
}
__host__ __device__ inline int32_t vx(uint64_t p) { return (int32_t)(p & 0x1FFFFF); }
__host__ __device__ inline int32_t vy(uint64_t p) { return (int32_t)((p >> 21) & 0x1FFFFF); }
__host__ __device__ inline int32_t vz(uint64_t p) { return (int32_t)((p >> 42) & 0x1FFFFF); }
__host__ __device__ inline uint64_t vmid(uint64_t a, uint64_t b) {
  return pack_vertex((vx(a) + vx(b)) >> 1, (vy(a) + vy(b)) >> 1, (vz(a) + vz(b)) >> 1);
}

// depth of a heap id: roots 8..13 (4 bits) are depth 0
__host__ __device__ inline int id_depth(uint64_t id) {
#if defined(__HIP_DEVICE_COMPILE__)
  return 60 - __clzll(id);
#else
  return 60 - __builtin_clzll(id);
#endif
}
__host__ __device__ inline int tag_of(int depth) { return 3 - depth % 3; }

// Depth-first keys are id << (60 - depth), so a key's top 4 bits are its
// root (8..13).  Bucket b of the key index holds the keys whose bits
// 63..60-kbits, less 8 << kbits, equal b (6 << kbits buckets); kidx[b] is
// the first index whose key is in bucket b or later, kidx[6 << kbits] = n.
__host__ __device__ inline int64_t key_buckets(int kbits) { return 6ll << kbits; }

// Last index whose key is <= key (-1 if none), searched within key's bucket.
__device__ inline int64_t search_keys_idx(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ kidx,
                                          int kbits, uint64_t key) {
  const uint64_t b = (key >> (60 - kbits)) - (8ull << kbits);
  int64_t lo = (int64_t)kidx[b] - 1, hi = kidx[b + 1];
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Shape classes.  Up to translation and scale every tet of these grids is
// one of a small set of shapes (with vertex order and tag): its edge
// vectors x_j - x_0 divided by their common power of two.  shape_table()
// gives the current device's table: word c (c < kShapeWords) describes
// class c: its bisection normal as a sign vector facing x_0 (bits 2i, 2i+1
// hold u_i + 1) and the classes of its first and second child (bits 8..15,
// 16..23); words kShapeWords + r hold the classes of the six roots.  Null
// if the table could not be made.
constexpr int kShapeWords = 256;
const uint32_t* shape_table();
// The current device's table if it has been made, else NULL (never allocates).
const uint32_t* shape_table_existing();

// Midpoint z of the edge (v0, vK) and the bisection normal of class word w.
template <int K>
__device__ inline void shape_bisector(const int32_t v[4][3], uint32_t w, int32_t z[3], int32_t u[3]) {
#pragma unroll
  for (int i = 0; i < 3; i++) {
    z[i] = (v[0][i] + v[K][i]) >> 1;
    u[i] = (int32_t)((w >> (2 * i)) & 3u) - 1;
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ inline uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// 24-bit uniform in [0,1) from a 32-bit word.
__device__ inline float u01(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// Draw `draw` of a stream: counter (pixel, sample, bounce << 8 | stream,
// draw >> 2), word draw & 3.
__device__ inline float uniform01(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t stream,
                                  uint32_t draw) {
  uint4 r = philox10(make_uint4(pixel, sample, (bounce << 8) | stream, draw >> 2), (uint32_t)seed,
                     (uint32_t)(seed >> 32));
  uint32_t w = (draw & 3) == 0 ? r.x : (draw & 3) == 1 ? r.y : (draw & 3) == 2 ? r.z : r.w;
  return u01(w);
}

// Words of draws `draw` and `draw + 1` (draw & 3 < 3: one Philox block).
__device__ inline uint2 uniform01x2(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t stream,
                                    uint32_t draw) {
  uint4 r = philox10(make_uint4(pixel, sample, (bounce << 8) | stream, draw >> 2), (uint32_t)seed,
                     (uint32_t)(seed >> 32));
  return (draw & 3) == 0 ? make_uint2(r.x, r.y) : ((draw & 3) == 1 ? make_uint2(r.y, r.z) : make_uint2(r.z, r.w));
}

enum { kStreamCamera = 0, kStreamFlight = 1, kStreamPhase = 2, kStreamLight = 3 };

// ---- elementary functions.  Each is evaluated in FP64 to about 1e-16
// relative accuracy and rounded once to FP32: the result is the correctly
// rounded value of the exact function unless that value lies within ~1e-16
// (relative) of the midpoint between two FP32 numbers.  They run per
// collision, scattering or light ray, never per walk step, and are called
// rather than inlined: their FP64 constants and temporaries then stay out of
// the tracing loop's register allocation (94 -> 82 VGPRs, no SGPR spills;
// tracing kernel 48.5 -> 47.7 ms on the cloud frame).

// -ln(1 - u) for u in [0, 1) (1 - u is exact in FP32): with 1 - u = m 2^e,
// m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s), s = (m - 1) / (m + 1),
// |s| <= 0.1716, by the atanh series through s^21 (truncation < 1e-17
// relative); ln(1 - u) = e ln 2 + ln m.
__device__ __attribute__((noinline)) float exp_tau(float u) {
  const float y = 1.0f - u;
  const uint32_t b = __float_as_uint(y);
  int e = (int)((b >> 23) & 0xFFu) - 127;
  double m = (double)__uint_as_float((b & 0x7FFFFFu) | 0x3F800000u);
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = p * z + 1.0 / 19.0;
  p = p * z + 1.0 / 17.0;
  p = p * z + 1.0 / 15.0;
  p = p * z + 1.0 / 13.0;
  p = p * z + 1.0 / 11.0;
  p = p * z + 1.0 / 9.0;
  p = p * z + 1.0 / 7.0;
  p = p * z + 1.0 / 5.0;
  p = p * z + 1.0 / 3.0;
  p = p * z + 1.0;
  const double lnm = (2.0 * s) * p;
  return (float)(0.0 - ((double)e * 0.6931471805599453 + lnm));
}

// e^-x for x >= 0 (0 from x >= 104 on, where the FP32 result rounds to 0):
// x = k ln 2 + r with k = rint(x / ln 2), ln 2 split in a 32-bit head (k ln2_hi
// exact) and a tail, |r| <= 0.347; e^-r by its Taylor polynomial through
// degree 13 (truncation < 5e-18), times 2^-k.
__device__ __attribute__((noinline)) float exp_neg(float x) {
  if (!(x < 104.0f)) return 0.0f;
  const double xd = (double)x;
  const double k = rint(xd * 1.4426950408889634);
  const double r = (xd - k * 0x1.62e42ffp-1) - k * -0x1.718432a1b0e26p-35;
  const double y = 0.0 - r;
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = p * y + 1.0 / 479001600.0;
  p = p * y + 1.0 / 39916800.0;
  p = p * y + 1.0 / 3628800.0;
  p = p * y + 1.0 / 362880.0;
  p = p * y + 1.0 / 40320.0;
  p = p * y + 1.0 / 5040.0;
  p = p * y + 1.0 / 720.0;
  p = p * y + 1.0 / 120.0;
  p = p * y + 1.0 / 24.0;
  p = p * y + 1.0 / 6.0;
  p = p * y + 0.5;
  p = p * y + 1.0;
  p = p * y + 1.0;
  return (float)ldexp(p, -(int)k);
}

// (cos, sin)(2 pi u) for u in [0, 1): quadrant q = round(4u), w = u - q/4
// (exact), theta = 2 pi w in FP64 (|theta| <= pi/4), Taylor polynomials
// through degree 18 / 17 (truncation < 1e-19), rotated by q.
__device__ __attribute__((noinline)) void sincos_2pi(float u, float& c, float& s) {
  const int q = (int)(u * 4.0f + 0.5f);
  const float w = u - (float)q * 0.25f;
  const double th = (double)w * 6.283185307179586;
  const double z = th * th;
  double ps = 1.0 / 355687428096000.0;  // 1/17!
  ps = ps * z - 1.0 / 1307674368000.0;
  ps = ps * z + 1.0 / 6227020800.0;
  ps = ps * z - 1.0 / 39916800.0;
  ps = ps * z + 1.0 / 362880.0;
  ps = ps * z - 1.0 / 5040.0;
  ps = ps * z + 1.0 / 120.0;
  ps = ps * z - 1.0 / 6.0;
  ps = ps * z + 1.0;
  double pc = -1.0 / 6402373705728000.0;  // -1/18!
  pc = pc * z + 1.0 / 20922789888000.0;
  pc = pc * z - 1.0 / 87178291200.0;
  pc = pc * z + 1.0 / 479001600.0;
  pc = pc * z - 1.0 / 3628800.0;
  pc = pc * z + 1.0 / 40320.0;
  pc = pc * z - 1.0 / 720.0;
  pc = pc * z + 1.0 / 24.0;
  pc = pc * z - 0.5;
  pc = pc * z + 1.0;
  const float sn = (float)(th * ps), cs = (float)pc;
  const int r = q & 3;
  c = r == 0 ? cs : (r == 1 ? 0.0f - sn : (r == 2 ? 0.0f - cs : sn));
  s = r == 0 ? sn : (r == 1 ? cs : (r == 2 ? 0.0f - sn : 0.0f - cs));
}

// Henyey-Greenstein density of the cosine mu between successive propagation
// directions, (1 - g^2) / (4 pi (1 + g^2 - 2 g mu)^(3/2)), in FP64 (IEEE
// division and square root), rounded once.
__device__ __attribute__((noinline)) float hg_pdf(float g, float mu) {
  const double gd = (double)g, md = (double)mu;
  const double g2 = gd * gd;
  const double den = (1.0 + g2) - (2.0 * gd) * md;
  return (float)((1.0 - g2) / (((4.0 * 3.141592653589793) * den) * sqrt(den)));
}

// Inverse HG cumulative distribution (isotropic limit 2u - 1 for
// |g| < 1e-3), in FP64, clamped to [-1, 1], rounded once.
__device__ __attribute__((noinline)) float hg_mu(float g, float u) {
  const double gd = (double)g, ud = (double)u;
  double mu;
  if (fabs(gd) < 1e-3) {
    mu = 2.0 * ud - 1.0;
  } else {
    const double g2 = gd * gd;
    const double sv = (1.0 - g2) / ((1.0 - gd) + (2.0 * gd) * ud);
    mu = ((1.0 + g2) - sv * sv) / (2.0 * gd);
  }
  mu = mu < -1.0 ? -1.0 : (mu > 1.0 ? 1.0 : mu);
  return (float)mu;
}

__device__ inline float3 normalize3(float3 v) {
  float l = sqrtf((v.x * v.x + v.y * v.y) + v.z * v.z);
  return make_float3(v.x / l, v.y / l, v.z / l);
}

// Scattered direction around d: polar cosine from HG, azimuth 2 pi u2, in
// the branchless orthonormal basis of Duff et al. (2017).
__device__ inline float3 hg_scatter(float3 d, float g, float u1, float u2) {
  float mu = hg_mu(g, u1);
  float q = 1.0f - mu * mu;
  q = q < 0.0f ? 0.0f : q;
  float st = sqrtf(q);
  float cp, sp;
  sincos_2pi(u2, cp, sp);
  float sign = copysignf(1.0f, d.z);
  float a = -1.0f / (sign + d.z);
  float b = (d.x * d.y) * a;
  float3 t1 = make_float3(1.0f + ((sign * d.x) * d.x) * a, sign * b, -sign * d.x);
  float3 t2 = make_float3(b, sign + (d.y * d.y) * a, -d.y);
  float ca = st * cp, cb = st * sp;
  float3 o = make_float3((t1.x * ca + t2.x * cb) + d.x * mu, (t1.y * ca + t2.y * cb) + d.y * mu,
                         (t1.z * ca + t2.z * cb) + d.z * mu);
  return normalize3(o);
}

// ---------------------------------------------------------------- host side
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

// Device-memory cache: blocks freed by the library are kept for reuse.
void* dev_alloc(size_t bytes);
void dev_free(void* p);

#define TV_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return ::tv::fail(TET_ERR_DEVICE, std::string(#call) + ": " +   \
                                            hipGetErrorString(e_));                        \
  } while (0)

// Camera frame / criterion quantities computed on the host in FP64.
void make_frame(const tet_camera& c, Frame* fr);
void make_camcrit(const tet_camera& c, float target_px, CamCrit* cc);
int check_camera(const tet_camera* c);

}  // namespace tv

struct tet_grid {
  int device;
  int64_t n;
  int32_t max_depth;
  int32_t majorant_mode;  // of the build (0 tight, 1 loose)
  tet_build_stats stats;
  uint64_t* ids;    // heap ids, depth-first order
  uint64_t* keys;   // depth-first keys (sorted ascending)
  uint32_t* kidx;   // bucket index of the keys (key_bucket_index)
  int32_t kbits;
  uint64_t* verts;  // 4 packed lattice vertices per tet
  uint64_t* chain;  // per tet: bit d = its depth-d ancestor was split because the want predicate held
  tv::TetRec* rec;      // traversal records
  tv::TetRec32* rec32;  // compact records (NULL when the grid cannot use them)
  float* ch[3];         // extra channels per tet: temperature, albedo, g (NULL = absent)
  // density model inside the tets: 0 constant (the records' extinction),
  // 1 linear (coefficients c0, gx, gy, gz per tet), 2 voxel lookup (a copy
  // of the volume); model records carry the model's majorant as extinction
  int32_t model;
  float* mmaj;
  float4* mcoef;
  float* mdens;
  int32_t mn;
  float mscale;
  tv::TetRec* mrec;
  tv::TetRec32* mrec32;
};
