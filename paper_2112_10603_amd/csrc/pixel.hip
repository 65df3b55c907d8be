// Per-pixel passes of the view-interpolation network: ingest and padding,
// the image pyramid, stage input assembly with flow upscaling and backward
// warps (Eq. 2), the final warp and mask blend (Eq. 1), the flow pyramid and
// the context-feature warps of the refinement U-Net, and the output head.
//
// All are memory-bound: one thread per output pixel (or per 8-channel group
// of a pixel), NHWC so the threads of a wavefront touch consecutive pixels.
// Sample positions, bilinear weights, flows and the mask stay fp32 in every
// precision; only the activations fed to convolutions use the activation
// dtype.
#include <type_traits>

#include "common.h"

namespace ffv {

namespace {

constexpr int TPB = 256;

template <typename T>
__device__ inline T cvt(float v) {
  return (T)v;
}

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// 16-byte packing of activation values: N values (N a multiple of 8 for
// bf16, of 4 for fp32) written to dst with 16-byte stores (dst 16-byte
// aligned), and 8 values read back with one or two 16-byte loads.
__device__ inline uint32_t pack2(float a, float b) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (bf16)a) | ((uint32_t)__builtin_bit_cast(uint16_t, (bf16)b) << 16);
}

template <typename T, int N>
__device__ inline void store_vals(T* dst, const float (&v)[N]) {
  if constexpr (sizeof(T) == 2) {
    static_assert(N % 8 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int k = 0; k < N; k += 8)
      *reinterpret_cast<uint4*>(dst + k) =
          make_uint4(pack2(v[k], v[k + 1]), pack2(v[k + 2], v[k + 3]), pack2(v[k + 4], v[k + 5]),
                     pack2(v[k + 6], v[k + 7]));
  } else {
    static_assert(N % 4 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int k = 0; k < N; k += 4)
      *reinterpret_cast<float4*>(dst + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
  }
}

// N values as 16-byte chunks in the layout store_vals writes.
template <typename T, int N>
__device__ inline void pack_chunks(const float (&v)[N], uint4 (&c)[N * sizeof(T) / 16]) {
  if constexpr (sizeof(T) == 2) {
    static_assert(N % 8 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int k = 0; k < N; k += 8)
      c[k / 8] = make_uint4(pack2(v[k], v[k + 1]), pack2(v[k + 2], v[k + 3]), pack2(v[k + 4], v[k + 5]),
                            pack2(v[k + 6], v[k + 7]));
  } else {
    static_assert(N % 4 == 0, "whole 16-byte chunks");
#pragma unroll
    for (int k = 0; k < N; k += 4)
      c[k / 4] = make_uint4(__float_as_uint(v[k]), __float_as_uint(v[k + 1]), __float_as_uint(v[k + 2]),
                            __float_as_uint(v[k + 3]));
  }
}

// Wave-contiguous stores of per-pixel records through LDS. The 64 lanes of a
// wave hold the NC-chunk records of 64 consecutive pixels, contiguous in
// memory. Stored lane by lane, each store instruction covers one chunk in NC
// of the wave's span, so every line is written in NC partial pieces and the
// write requests multiply by NC (measured: the 48-byte records of the stage
// transition took 5.5 of its 8.6 ms at 1080p x 112 views). Instead each lane
// puts its record into the wave's LDS area (stage_put), the block meets at a
// barrier, and each store instruction then writes 64 consecutive chunks
// (stage_flush); records of pixels at or past the last valid one are not
// written. These stores, and the final pass's blended image, are marked
// non-temporal: a pass streams out far more than the caches hold, so
// keeping its output lines cached only evicts the camera rows and flow
// taps its waves are still gathering (measured at 1080p x 112 views: final
// pass 8.96 -> 8.38 ms, stage transitions 9.04 -> 8.71 ms, the kernels
// that read the records unchanged).
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ inline void store_nt(uint4* dst, const uint4& w) {
  const u32x4 v = {w.x, w.y, w.z, w.w};
  __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(dst));
}

__device__ inline void store_nt(float* dst, const float4& w) {
  const f32x4 v = {w.x, w.y, w.z, w.w};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst));
}

template <int NC>
__device__ inline void stage_put(uint4* wave_stage, int lane, const uint4 (&c)[NC]) {
#pragma unroll
  for (int k = 0; k < NC; ++k) wave_stage[lane * NC + k] = c[k];
}

template <int NC>
__device__ inline void stage_flush(const uint4* wave_stage, int lane, uint4* dst, int n_valid) {
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = k * 64 + lane;
    if (c / NC < n_valid) store_nt(dst + c, wave_stage[c]);
  }
}

template <typename T>
__device__ inline void load8(const T* src, float (&v)[8]) {
  if constexpr (sizeof(T) == 2) {
    const uint4 u = *reinterpret_cast<const uint4*>(src);
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = __uint_as_float(w[k] << 16);
      v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
  } else {
    const float4 a = *reinterpret_cast<const float4*>(src), b = *reinterpret_cast<const float4*>(src + 4);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
  }
}

// Workgroup order of a (pixel blocks x views) grid for the final warp and
// blend. Consecutive workgroup ids go to the 8 XCDs in turn, each with its
// own L2; every XCD instead takes a contiguous range of an order that
// visits one pixel block of every view before the next block, so the views
// of a camera pair running together on an XCD read the same camera rows
// from its L2. (Measured: 11 % faster for the final pass at 1080p x 112
// views; the stage transition, whose output streams are wider, and the
// other passes measured equal or slower with it.)
__device__ inline void view_fastest_order(long& bx, int& v) {
  const unsigned long gx = gridDim.x, gy = gridDim.y;
  const unsigned long total = gx * gy;
  const unsigned long id = (unsigned long)blockIdx.y * gx + blockIdx.x;
  const unsigned long q = total >> 3, r = total & 7, x = id & 7;
  const unsigned long lg = x * q + (x < r ? x : r) + (id >> 3);
  bx = (long)(lg / gy);
  v = (int)(lg - (unsigned long)bx * gy);
}

// Workgroup order within one image of a (pixel blocks x images) grid, for
// passes that read a pixel's neighbours (3x3 taps, bilinear warp and
// upsampling taps). Consecutive workgroup ids go to the 8 XCDs in turn,
// each with its own L2, so in launch order the block below a block (one
// row of 1920 pixels is 7.5 blocks) runs on another XCD and every row is
// fetched into several L2s. Here the blocks that land on one XCD take a
// contiguous band of the image instead, while all XCDs still work on the
// same image at the same time (its cameras' rows stay shared in the
// last-level cache). Measured at 1080p x 112 views: L2 misses of the
// context warps fall 3.3x and of the head 2.1x, for 5-15 % and 2 % less
// time (these passes wait on latency more than on bytes); the stage
// transition, whose record writes dominate, runs 10 % slower with it and
// keeps the launch order.
__device__ inline long banded_block() {
  const unsigned gx = gridDim.x, i = blockIdx.x;
  // the blocks of this image with the same id mod 8 share an XCD
  const unsigned r = i & 7u, q = gx >> 3, rem = gx & 7u;
  return (long)(r * q + (r < rem ? r : rem) + (i >> 3));
}

// Half-pixel-centre source coordinate for resampling n_in -> n_out.
__device__ inline void hp_tap(int i, int n_in, int n_out, int& i0, int& i1, float& w) {
  float s = ((float)i + 0.5f) * ((float)n_in / (float)n_out) - 0.5f;
  s = fmaxf(s, 0.f);
  int f = (int)floorf(s);
  if (f > n_in - 1) f = n_in - 1;
  i0 = f;
  i1 = min(f + 1, n_in - 1);
  w = s - (float)f;
}

// Backward bilinear sample position u + f, clamped to the image (border mode).
struct Tap4 {
  int o00, o01, o10, o11;  // pixel offsets
  float w00, w01, w10, w11;
};

__device__ inline Tap4 warp_taps(int x, int y, float fx, float fy, int w, int h) {
  float px = fminf(fmaxf((float)x + fx, 0.f), (float)(w - 1));
  float py = fminf(fmaxf((float)y + fy, 0.f), (float)(h - 1));
  int x0 = (int)floorf(px), y0 = (int)floorf(py);
  int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
  float a = px - (float)x0, b = py - (float)y0;
  Tap4 t;
  t.o00 = y0 * w + x0;
  t.o01 = y0 * w + x1;
  t.o10 = y1 * w + x0;
  t.o11 = y1 * w + x1;
  t.w00 = (1.f - a) * (1.f - b);
  t.w01 = a * (1.f - b);
  t.w10 = (1.f - a) * b;
  t.w11 = a * b;
  return t;
}

__device__ inline float4 sample4(const float* img, const Tap4& t) {
  float4 p00 = ld4(img + 4L * t.o00), p01 = ld4(img + 4L * t.o01);
  float4 p10 = ld4(img + 4L * t.o10), p11 = ld4(img + 4L * t.o11);
  float4 r;
  r.x = t.w00 * p00.x + t.w01 * p01.x + t.w10 * p10.x + t.w11 * p11.x;
  r.y = t.w00 * p00.y + t.w01 * p01.y + t.w10 * p10.y + t.w11 * p11.y;
  r.z = t.w00 * p00.z + t.w01 * p01.z + t.w10 * p10.z + t.w11 * p11.z;
  r.w = 0.f;
  return r;
}

// ---------------------------------------------------------------- ingest
template <typename T>
__global__ void ingest_k(const float* const* src, int H, int W, int Hp, int Wp, float* X4, T* Xa) {
  const int cam = blockIdx.y;
  const long P = (long)Hp * Wp;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= P) return;
  const int y = (int)(p / Wp), x = (int)(p % Wp);
  const int sy = min(y, H - 1), sx = min(x, W - 1);
  const float* s = src[cam];
  const long HW = (long)H * W;
  const float r = s[(long)sy * W + sx], g = s[HW + (long)sy * W + sx], b = s[2 * HW + (long)sy * W + sx];
  *reinterpret_cast<float4*>(X4 + (cam * P + p) * 4) = make_float4(r, g, b, 0.f);
  const float xv[8] = {r, g, b, 0.f, 0.f, 0.f, 0.f, 0.f};
  store_vals<T, 8>(Xa + (cam * P + p) * 8, xv);
}

// ----------------------------------------------------- 4-channel resample
__global__ void resample4_k(const float* in, int Hi, int Wi, float* out, int Ho, int Wo) {
  const int img = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= (long)Ho * Wo) return;
  const int y = (int)(p / Wo), x = (int)(p % Wo);
  int y0, y1, x0, x1;
  float by, ax;
  hp_tap(y, Hi, Ho, y0, y1, by);
  hp_tap(x, Wi, Wo, x0, x1, ax);
  const float* b = in + (long)img * Hi * Wi * 4;
  float4 a00 = ld4(b + 4L * (y0 * Wi + x0)), a01 = ld4(b + 4L * (y0 * Wi + x1));
  float4 a10 = ld4(b + 4L * (y1 * Wi + x0)), a11 = ld4(b + 4L * (y1 * Wi + x1));
  float4 r;
  r.x = (a00.x * (1.f - ax) + a01.x * ax) * (1.f - by) + (a10.x * (1.f - ax) + a11.x * ax) * by;
  r.y = (a00.y * (1.f - ax) + a01.y * ax) * (1.f - by) + (a10.y * (1.f - ax) + a11.y * ax) * by;
  r.z = (a00.z * (1.f - ax) + a01.z * ax) * (1.f - by) + (a10.z * (1.f - ax) + a11.z * ax) * by;
  r.w = (a00.w * (1.f - ax) + a01.w * ax) * (1.f - by) + (a10.w * (1.f - ax) + a11.w * ax) * by;
  *reinterpret_cast<float4*>(out + ((long)img * Ho * Wo + p) * 4) = r;
}

// ------------------------------------------------------ stage-0 input
template <typename T>
__global__ void assemble0_k(const ViewDesc* views, const CamDev* cams, int h, int w, T* x, int ld,
                            int t_plane) {
  const int v = blockIdx.y;
  const long P = (long)h * w;  // slot stride
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  const ViewDesc d = views[v];
  if (p >= (long)(d.hp >> 2) * (d.wp >> 2)) return;
  const float4 l = ld4(cams[d.cam_l].L0 + 4 * p);
  const float4 r = ld4(cams[d.cam_r].L0 + 4 * p);
  const float vals[8] = {l.x, l.y, l.z, r.x, r.y, r.z, t_plane ? d.t : 0.f, 0.f};
  store_vals<T, 8>(x + ((long)v * P + p) * ld, vals);
}

// ---------------------------------------- stage transition s -> s+1 (Eq. 2)
// FM layout: 8 floats per pixel = (F_l.x, F_l.y, F_r.x, F_r.y, M, 0, 0, 0).
template <typename T>
__global__ __launch_bounds__(TPB) void transition_k(const ViewDesc* views, const CamDev* cams, int level,
                                                    const float* FMprev, int hp, int wp, int h, int w, T* x,
                                                    int ld, float* FM, int t_plane) {
  constexpr int NX = 24 * (int)sizeof(T) / 16;  // chunks of a pixel's 24 activations
  __shared__ uint4 stage[TPB * (NX + 2)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v = blockIdx.y;
  const long bx = blockIdx.x;  // launch order: measured faster here than banded_block()
  const long P = (long)h * w;  // slot strides: P here, hp * wp for the previous level
  const ViewDesc d = views[v];
  const int vh = d.hp >> (2 - level), vw = d.wp >> (2 - level);  // this view's level sizes
  const int vhp = vh >> 1, vwp = vw >> 1;
  const long n_px = (long)vh * vw;
  const long p0 = bx * TPB + wave * 64;  // the wave's first pixel
  if (bx * TPB >= n_px) return;  // uniform over the block
  // lanes past the view's last pixel compute pixel 0 and store nothing
  const long p = p0 + lane < n_px ? p0 + lane : 0;
  const int y = (int)(p / vw), xx = (int)(p % vw);
  int y0, y1, x0, x1;
  float by, ax;
  hp_tap(y, vhp, vh, y0, y1, by);
  hp_tap(xx, vwp, vw, x0, x1, ax);
  const float* fp = FMprev + (long)v * hp * wp * 8;
  const float* q00 = fp + 8L * (y0 * vwp + x0);
  const float* q01 = fp + 8L * (y0 * vwp + x1);
  const float* q10 = fp + 8L * (y1 * vwp + x0);
  const float* q11 = fp + 8L * (y1 * vwp + x1);
  float up[5];
#pragma unroll
  for (int c = 0; c < 5; ++c)
    up[c] = (q00[c] * (1.f - ax) + q01[c] * ax) * (1.f - by) + (q10[c] * (1.f - ax) + q11[c] * ax) * by;
  const float Fx = 2.f * up[0], Fy = 2.f * up[1], Gx = 2.f * up[2], Gy = 2.f * up[3], Mt = up[4];

  const float* Lc = level == 1 ? cams[d.cam_l].L1 : cams[d.cam_l].X4;
  const float* Rc = level == 1 ? cams[d.cam_r].L1 : cams[d.cam_r].X4;
  const float4 L = ld4(Lc + 4 * p), R = ld4(Rc + 4 * p);
  const float4 Wl = sample4(Lc, warp_taps(xx, y, Fx, Fy, vw, vh));
  const float4 Wr = sample4(Rc, warp_taps(xx, y, Gx, Gy, vw, vh));

  const float vals[24] = {L.x, L.y, L.z, R.x, R.y, R.z, Wl.x, Wl.y, Wl.z, Wr.x, Wr.y, Wr.z,
                          Mt, Fx, Fy, Gx, Gy, t_plane ? d.t : 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uint4 cx[NX];
  pack_chunks<T, 24>(vals, cx);
  const uint4 cf[2] = {make_uint4(__float_as_uint(Fx), __float_as_uint(Fy), __float_as_uint(Gx), __float_as_uint(Gy)),
                       make_uint4(__float_as_uint(Mt), 0u, 0u, 0u)};
  uint4* sx = stage + wave * 64 * NX;
  uint4* sf = stage + TPB * NX + wave * 128;
  stage_put<NX>(sx, lane, cx);
  stage_put<2>(sf, lane, cf);
  __syncthreads();
  const int n_valid = (int)(n_px - p0 < 64 ? n_px - p0 : 64);
  stage_flush<NX>(sx, lane, reinterpret_cast<uint4*>(x + ((long)v * P + p0) * ld), n_valid);
  stage_flush<2>(sf, lane, reinterpret_cast<uint4*>(FM + ((long)v * P + p0) * 8), n_valid);
}

// ------------------------------------ final warp + mask blend (Eq. 1)
template <typename T>
__global__ __launch_bounds__(TPB) void final_k(const ViewDesc* views, const CamDev* cams, const float* FM,
                                               int h, int w, float* I2, T* x0u, int ld) {
  constexpr int NX = 24 * (int)sizeof(T) / 16;  // chunks of a pixel's 24 activations
  __shared__ uint4 stage[TPB * NX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long bx;
  int v;
  view_fastest_order(bx, v);
  const long P = (long)h * w;  // slot stride
  const ViewDesc d = views[v];
  const int vh = d.hp, vw = d.wp;  // this view's size
  const long n_px = (long)vh * vw;
  const long p0 = bx * TPB + wave * 64;  // the wave's first pixel
  if (bx * TPB >= n_px) return;  // uniform over the block
  // lanes past the view's last pixel compute pixel 0 and store nothing
  const bool in = p0 + lane < n_px;
  const long p = in ? p0 + lane : 0;
  const int y = (int)(p / vw), xx = (int)(p % vw);
  const float* f = FM + ((long)v * P + p) * 8;
  const float4 F = ld4(f);
  const float M = f[4];
  const float* Lc = cams[d.cam_l].X4;
  const float* Rc = cams[d.cam_r].X4;
  const float4 L = ld4(Lc + 4 * p), R = ld4(Rc + 4 * p);
  const float4 Wl = sample4(Lc, warp_taps(xx, y, F.x, F.y, vw, vh));
  const float4 Wr = sample4(Rc, warp_taps(xx, y, F.z, F.w, vw, vh));
  const float m = 1.f / (1.f + expf(-M));
  float4 o;
  o.x = m * Wl.x + (1.f - m) * Wr.x;
  o.y = m * Wl.y + (1.f - m) * Wr.y;
  o.z = m * Wl.z + (1.f - m) * Wr.z;
  o.w = 0.f;
  if (in) store_nt(I2 + ((long)v * P + p) * 4, o);
  const float vals[24] = {L.x, L.y, L.z, R.x, R.y, R.z, Wl.x, Wl.y, Wl.z, Wr.x, Wr.y, Wr.z,
                          M, F.x, F.y, F.z, F.w, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uint4 cx[NX];
  pack_chunks<T, 24>(vals, cx);
  uint4* sx = stage + wave * 64 * NX;
  stage_put<NX>(sx, lane, cx);
  __syncthreads();
  const int n_valid = (int)(n_px - p0 < 64 ? n_px - p0 : 64);
  stage_flush<NX>(sx, lane, reinterpret_cast<uint4*>(x0u + ((long)v * P + p0) * ld), n_valid);
}

// ------------------------------- blend-only output (no refinement, Table 1)
// out = I2, cropped to H x W and written planar [3][H][W].
__global__ void blend_out_k(const float* I2, const ViewDesc* views, int Hp, int Wp, int H, int W) {
  const int v = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  const ViewDesc d = views[v];
  if (p >= (long)d.h * d.w) return;
  const int y = (int)(p / d.w), x = (int)(p % d.w);
  const float4 b = ld4(I2 + ((long)v * Hp * Wp + (long)y * d.wp + x) * 4);
  const long HW = (long)d.h * d.w;
  float* o = d.out;
  o[p] = b.x;
  o[HW + p] = b.y;
  o[2 * HW + p] = b.z;
}

// -------------------------------------------- flow pyramid: F/2 of 2x2 mean
__global__ void flow_down_k(const float* in, int in_ld, const ViewDesc* views, int k, int h, int w, float* out) {
  const int img = blockIdx.y;
  const long bx = banded_block();
  const int ho = h / 2, wo = w / 2;  // slot strides: h x w in, ho x wo out
  const long p = bx * TPB + threadIdx.x;
  const ViewDesc d = views[img];
  const int vw = d.wp >> k;  // this view's level-k width
  const int vwo = vw >> 1;
  if (p >= (long)((d.hp >> k) >> 1) * vwo) return;
  const int y = (int)(p / vwo), x = (int)(p % vwo);
  const float* b = in + (long)img * h * w * in_ld;
  const float4 a = ld4(b + (long)in_ld * ((2 * y) * vw + 2 * x));
  const float4 c = ld4(b + (long)in_ld * ((2 * y) * vw + 2 * x + 1));
  const float4 e = ld4(b + (long)in_ld * ((2 * y + 1) * vw + 2 * x));
  const float4 g = ld4(b + (long)in_ld * ((2 * y + 1) * vw + 2 * x + 1));
  float4 r;
  r.x = 0.5f * (0.5f * (0.5f * (a.x + c.x) + 0.5f * (e.x + g.x)));
  r.y = 0.5f * (0.5f * (0.5f * (a.y + c.y) + 0.5f * (e.y + g.y)));
  r.z = 0.5f * (0.5f * (0.5f * (a.z + c.z) + 0.5f * (e.z + g.z)));
  r.w = 0.5f * (0.5f * (0.5f * (a.w + c.w) + 0.5f * (e.w + g.w)));
  *reinterpret_cast<float4*>(out + ((long)img * ho * wo + p) * 4) = r;
}

// ------------------------------------------------ context-feature warp
// One thread per (pixel, 8-channel group); groups [0, C/8) warp the left
// camera's features by F_l, groups [C/8, C/4) the right's by F_r.
template <typename T>
__global__ void ctx_warp_k(const ViewDesc* views, const CamDev* cams, int level, int C,
                           const float* flow, int h, int w, T* dst, int dst_ld, long dst_img_stride) {
  const int v = blockIdx.y;
  const long bx = banded_block();
  const int G = C / 4;  // groups for both sides
  const long P = (long)h * w;  // slot stride
  const long id = bx * TPB + threadIdx.x;
  const ViewDesc d = views[v];
  const int vh = d.hp >> (level + 1), vw = d.wp >> (level + 1);  // this view's level size
  if (id >= (long)vh * vw * G) return;
  const long p = id / G;
  const int g = (int)(id - p * G);
  const bool right = g >= G / 2;
  const int c0 = (right ? g - G / 2 : g) * 8;
  const int y = (int)(p / vw), x = (int)(p % vw);
  const float4 F = ld4(flow + ((long)v * P + p) * 4);
  const Tap4 t = right ? warp_taps(x, y, F.z, F.w, vw, vh) : warp_taps(x, y, F.x, F.y, vw, vh);
  const T* src = reinterpret_cast<const T*>(cams[right ? d.cam_r : d.cam_l].ctx[level]) + c0;
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
  const int offs[4] = {t.o00, t.o01, t.o10, t.o11};
  const float ws[4] = {t.w00, t.w01, t.w10, t.w11};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float a[8];
    load8<T>(src + (long)offs[q] * C, a);
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += ws[q] * a[i];
  }
  store_vals<T, 8>(dst + (long)v * dst_img_stride + p * dst_ld + (right ? C : 0) + c0, acc);
}

// ----------------------------------------------------------- output head
// r = sigmoid(conv3x3(u4 -> 3)); out = clamp(I2 + 2r - 1, 0, 1), cropped and
// written planar [3][H][W]. C (the U-Net's last width) is a multiple of 8,
// at most 64, and a template parameter: each tap's C channels arrive as
// 16-byte vector loads, and the three output weights of a (tap, channel)
// are one float4 in LDS (the same address in every lane: a broadcast).
template <typename T>
__device__ inline void load_chunk(const T* p, float (&v)[16 / sizeof(T)]);

template <>
__device__ inline void load_chunk<bf16>(const bf16* p, float (&v)[8]) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = __uint_as_float(w[k] << 16);
    v[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}

template <>
__device__ inline void load_chunk<float>(const float* p, float (&v)[4]) {
  const float4 u = *reinterpret_cast<const float4*>(p);
  v[0] = u.x;
  v[1] = u.y;
  v[2] = u.z;
  v[3] = u.w;
}

template <typename T, int C>
__global__ void head_k(const T* u4, int ld, const float* wgt, const float* bias, const float* I2,
                       const ViewDesc* views, int Hp, int Wp, int H, int W) {
  constexpr int V = 16 / (int)sizeof(T);  // channels per 16-byte load
  static_assert(C % V == 0, "whole vector loads");
  __shared__ float4 ws[9 * C];  // [tap][channel] -> (w_r, w_g, w_b, 0)
  for (int i = threadIdx.x; i < 9 * C; i += TPB) {
    const int tap = i / C, c = i - tap * C;
    ws[i] = make_float4(wgt[(0 * C + c) * 9 + tap], wgt[(1 * C + c) * 9 + tap],
                        wgt[(2 * C + c) * 9 + tap], 0.f);
  }
  __syncthreads();
  const int v = blockIdx.y;
  const long bx = banded_block();
  const long p = bx * TPB + threadIdx.x;
  const ViewDesc d = views[v];
  if (p >= (long)d.h * d.w) return;
  const long slot = (long)v * Hp * Wp;  // slot stride of the launch's size
  // this view's size from here on
  H = d.h;
  W = d.w;
  Hp = d.hp;
  Wp = d.wp;
  const int y = (int)(p / W), x = (int)(p % W);
  const T* base = u4 + slot * ld;
  float z0 = bias[0], z1 = bias[1], z2 = bias[2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    if (yy < 0 || yy >= Hp || xx < 0 || xx >= Wp) continue;  // zero padding
    const T* s = base + ((long)yy * Wp + xx) * ld;
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += V) {
      float a[V];
      load_chunk<T>(s + c0, a);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const float4 w = ws[tap * C + c0 + k];
        z0 += w.x * a[k];
        z1 += w.y * a[k];
        z2 += w.z * a[k];
      }
    }
  }
  const float4 b = ld4(I2 + (slot + (long)y * Wp + x) * 4);
  const float r0 = 1.f / (1.f + expf(-z0)), r1 = 1.f / (1.f + expf(-z1)), r2 = 1.f / (1.f + expf(-z2));
  const long HW = (long)H * W;
  float* o = d.out;
  o[p] = fminf(fmaxf(b.x + 2.f * r0 - 1.f, 0.f), 1.f);
  o[HW + p] = fminf(fmaxf(b.y + 2.f * r1 - 1.f, 0.f), 1.f);
  o[2 * HW + p] = fminf(fmaxf(b.z + 2.f * r2 - 1.f, 0.f), 1.f);
}

// The same head for bf16 activations on the matrix cores: the 3x3 conv is a
// GEMM with the 3 output channels (zero-padded to 32) as the A operand and
// 32 pixels as B, K = (tap, channel) in 16-channel MFMA steps. A wave
// computes groups of 32 consecutive pixels of the crop: lane l reads, per
// tap, the 8 channels 8*(l/32).. of pixel l%32's neighbour (one 16-byte
// load), and ends with that pixel's three pre-activations in its first
// accumulators (lanes 0-31). The weights are rounded to bf16 (as every other
// bf16 layer's) and laid out once per block as MFMA fragments in LDS; a
// block covers HEAD_GROUPS groups per wave to amortise that.
constexpr int HEAD_GROUPS = 32;
// threads per block of the MFMA head: eight waves share one weight table
// (measured 6 % faster than four at 1080p x 112 views)
constexpr int HEAD_TPB = 512;

template <int C>
__global__ __launch_bounds__(HEAD_TPB) void head_mfma_k(const bf16* u4, int ld, const float* wgt,
                                                   const float* bias, const float* I2,
                                                   const ViewDesc* views, int Hp, int Wp, int H, int W) {
  constexpr int NC = C / 16;  // MFMAs per tap
  constexpr int WAVES = HEAD_TPB / 64;
  __shared__ uint4 wtab[9 * NC * 64];  // [tap][j][lane] weight fragments
  for (int i = threadIdx.x; i < 9 * NC * 64; i += HEAD_TPB) {
    const int ln = i & 63, tj = i >> 6, tap = tj / NC, j = tj - tap * NC;
    const int n = ln & 31, h = ln >> 5;
    bf16x8 w;
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = (bf16)(n < 3 ? wgt[(n * C + 16 * j + 8 * h + k) * 9 + tap] : 0.f);
    wtab[i] = __builtin_bit_cast(uint4, w);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lrow = lane & 31, lhalf = lane >> 5;
  const int v = blockIdx.y;
  const long bx = banded_block();
  const ViewDesc d = views[v];
  const long slot = (long)v * Hp * Wp;  // slot stride of the launch's size
  // this view's size from here on
  H = d.h;
  W = d.w;
  Hp = d.hp;
  Wp = d.wp;
  const long HW = (long)H * W;
  const bf16* base = u4 + slot * ld + 8 * lhalf;
  const float bias0 = bias[0], bias1 = bias[1], bias2 = bias[2];
  float* o = d.out;
  // One group per iteration: its nine tap loads and the blend input go out
  // together and wait for one memory round trip. (Two groups per
  // iteration halve the round trips but need 132 registers, three waves
  // per SIMD; one group keeps more waves resident and measured 16 % faster
  // at 1080p x 112 views.)
  for (int g = 0; g < HEAD_GROUPS; ++g) {
    if ((bx * HEAD_GROUPS + g) * WAVES * 32 >= HW) break;  // uniform over the block
    const long p = ((bx * HEAD_GROUPS + g) * WAVES + wave) * 32 + lrow;
    const bool pin = p < HW;
    const int y = pin ? (int)(p / W) : 0;
    const int x = pin ? (int)(p % W) : 0;
    uint4 av[9][NC];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      const bool ok = pin && yy >= 0 && yy < Hp && xx >= 0 && xx < Wp;  // zero padding
      const bf16* src = base + ((long)(ok ? yy : 0) * Wp + (ok ? xx : 0)) * ld;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        av[tap][j] = ok ? *reinterpret_cast<const uint4*>(src + 16 * j) : make_uint4(0u, 0u, 0u, 0u);
    }
    const float4 b = ld4(I2 + (slot + (long)y * Wp + x) * 4);
    f32x16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int j = 0; j < NC; ++j)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, wtab[(tap * NC + j) * 64 + lane]),
                                                      __builtin_bit_cast(bf16x8, av[tap][j]), acc, 0, 0, 0);
    if (lhalf == 0 && pin) {
      const float z0 = acc[0] + bias0, z1 = acc[1] + bias1, z2 = acc[2] + bias2;
      const float r0 = 1.f / (1.f + expf(-z0)), r1 = 1.f / (1.f + expf(-z1)), r2 = 1.f / (1.f + expf(-z2));
      o[p] = fminf(fmaxf(b.x + 2.f * r0 - 1.f, 0.f), 1.f);
      o[HW + p] = fminf(fmaxf(b.y + 2.f * r1 - 1.f, 0.f), 1.f);
      o[2 * HW + p] = fminf(fmaxf(b.z + 2.f * r2 - 1.f, 0.f), 1.f);
    }
  }
}

// -------------------------------------------------------- layout helpers
template <typename T>
__global__ void extract_k(const T* src, int ld, int C, long n_pix, float* dst) {
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= n_pix) return;
  for (int c = 0; c < C; ++c) dst[c * n_pix + p] = (float)src[p * ld + c];
}

template <typename T>
__global__ void pack_nhwc_k(const float* src, int C, int H, int W, T* dst, int ld) {
  const int img = blockIdx.y;
  const long P = (long)H * W;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= P) return;
  const float* s = src + (long)img * C * P;
  T* o = dst + ((long)img * P + p) * ld;
  for (int c = 0; c < ld; ++c) o[c] = cvt<T>(c < C ? s[c * P + p] : 0.f);
}

inline dim3 grid1(long n, int y) { return dim3((unsigned)((n + TPB - 1) / TPB), (unsigned)y); }

}  // namespace

#define FFV_DISPATCH(dt, KERNEL, ...)                                     \
  do {                                                                     \
    if ((dt) == DType::F32)                                                \
      hipLaunchKernelGGL(KERNEL<float>, __VA_ARGS__);                      \
    else                                                                   \
      hipLaunchKernelGGL(KERNEL<bf16>, __VA_ARGS__);                       \
  } while (0)

hipError_t launch_ingest(const float* const* src, int n_cam, int H, int W, int Hp, int Wp, float* X4,
                         void* Xa, DType dt, hipStream_t s) {
  if (n_cam <= 0) return hipSuccess;
  if (dt == DType::F32)
    hipLaunchKernelGGL(ingest_k<float>, grid1((long)Hp * Wp, n_cam), dim3(TPB), 0, s, src, H, W, Hp,
                       Wp, X4, (float*)Xa);
  else
    hipLaunchKernelGGL(ingest_k<bf16>, grid1((long)Hp * Wp, n_cam), dim3(TPB), 0, s, src, H, W, Hp,
                       Wp, X4, (bf16*)Xa);
  return hipGetLastError();
}

hipError_t launch_resample4(const float* in, int n_img, int Hi, int Wi, float* out, int Ho, int Wo,
                            hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(resample4_k, grid1((long)Ho * Wo, n_img), dim3(TPB), 0, s, in, Hi, Wi, out, Ho,
                     Wo);
  return hipGetLastError();
}

hipError_t launch_assemble0(const ViewDesc* views, int n_views, const CamDev* cams, int h, int w,
                            void* x, int ld, DType dt, int t_plane, hipStream_t s) {
  if (n_views <= 0) return hipSuccess;
  if (ld != 8) return hipErrorInvalidValue;  // one 16-byte-aligned run of 8 channels
  if (dt == DType::F32)
    hipLaunchKernelGGL(assemble0_k<float>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams,
                       h, w, (float*)x, ld, t_plane);
  else
    hipLaunchKernelGGL(assemble0_k<bf16>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams,
                       h, w, (bf16*)x, ld, t_plane);
  return hipGetLastError();
}

hipError_t launch_transition(const ViewDesc* views, int n_views, const CamDev* cams, int level,
                             const float* FMprev, int hp, int wp, int h, int w, void* x, int ld,
                             float* FM, DType dt, int t_plane, hipStream_t s) {
  if (n_views <= 0) return hipSuccess;
  if (ld != 24) return hipErrorInvalidValue;  // 18 channels padded to 24 (16-byte runs)
  if (dt == DType::F32)
    hipLaunchKernelGGL(transition_k<float>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams,
                       level, FMprev, hp, wp, h, w, (float*)x, ld, FM, t_plane);
  else
    hipLaunchKernelGGL(transition_k<bf16>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams,
                       level, FMprev, hp, wp, h, w, (bf16*)x, ld, FM, t_plane);
  return hipGetLastError();
}

hipError_t launch_final(const ViewDesc* views, int n_views, const CamDev* cams, const float* FM,
                        int h, int w, float* I2, void* x0u, int ld, DType dt, hipStream_t s) {
  if (n_views <= 0) return hipSuccess;
  if (ld != 24) return hipErrorInvalidValue;  // 17 channels padded to 24 (16-byte runs)
  if (dt == DType::F32)
    hipLaunchKernelGGL(final_k<float>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams, FM, h,
                       w, I2, (float*)x0u, ld);
  else
    hipLaunchKernelGGL(final_k<bf16>, grid1((long)h * w, n_views), dim3(TPB), 0, s, views, cams, FM, h,
                       w, I2, (bf16*)x0u, ld);
  return hipGetLastError();
}

hipError_t launch_flow_down(const float* in, int in_ld, const ViewDesc* views, int n_img, int k, int h, int w,
                            float* out, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(flow_down_k, grid1((long)(h / 2) * (w / 2), n_img), dim3(TPB), 0, s, in, in_ld, views, k,
                     h, w, out);
  return hipGetLastError();
}

hipError_t launch_ctx_warp(const ViewDesc* views, int n_views, const CamDev* cams, int level, int C,
                           const float* flow, int h, int w, void* dst, int dst_ld,
                           long dst_img_stride, DType dt, hipStream_t s) {
  if (n_views <= 0) return hipSuccess;
  // 8-channel groups as 16-byte loads and stores
  if (C % 8 != 0 || dst_ld % 8 != 0 || dst_img_stride % 8 != 0 ||
      reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return hipErrorInvalidValue;
  const long n = (long)h * w * (C / 4);
  if (dt == DType::F32)
    hipLaunchKernelGGL(ctx_warp_k<float>, grid1(n, n_views), dim3(TPB), 0, s, views, cams, level, C,
                       flow, h, w, (float*)dst, dst_ld, dst_img_stride);
  else
    hipLaunchKernelGGL(ctx_warp_k<bf16>, grid1(n, n_views), dim3(TPB), 0, s, views, cams, level, C,
                       flow, h, w, (bf16*)dst, dst_ld, dst_img_stride);
  return hipGetLastError();
}

hipError_t launch_head(const void* u4, int ld, int C, const float* w, const float* b,
                       const float* I2, const ViewDesc* views, int n_img, int Hp, int Wp, int H,
                       int W, DType dt, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  if (C <= 0 || C > 64 || C % 8 != 0 || C > ld || ld % 8 != 0) return hipErrorInvalidValue;
  if (dt == DType::BF16 && (C == 16 || C == 32)) {
    const long per_block = (long)HEAD_GROUPS * (HEAD_TPB / 64) * 32;  // groups of 32 pixels per wave
    const dim3 g((unsigned)(((long)H * W + per_block - 1) / per_block), (unsigned)n_img);
    if (C == 16)
      hipLaunchKernelGGL(head_mfma_k<16>, g, dim3(HEAD_TPB), 0, s, (const bf16*)u4, ld, w, b, I2, views, Hp, Wp,
                         H, W);
    else
      hipLaunchKernelGGL(head_mfma_k<32>, g, dim3(HEAD_TPB), 0, s, (const bf16*)u4, ld, w, b, I2, views, Hp, Wp,
                         H, W);
    return hipGetLastError();
  }
  const dim3 grid = grid1((long)H * W, n_img);
  auto go = [&](auto tc) {
    constexpr int CC = decltype(tc)::value;
    if (dt == DType::F32)
      hipLaunchKernelGGL((head_k<float, CC>), grid, dim3(TPB), 0, s, (const float*)u4, ld, w, b, I2, views,
                         Hp, Wp, H, W);
    else
      hipLaunchKernelGGL((head_k<bf16, CC>), grid, dim3(TPB), 0, s, (const bf16*)u4, ld, w, b, I2, views,
                         Hp, Wp, H, W);
  };
  switch (C) {
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 16: go(std::integral_constant<int, 16>{}); break;
    case 24: go(std::integral_constant<int, 24>{}); break;
    case 32: go(std::integral_constant<int, 32>{}); break;
    case 40: go(std::integral_constant<int, 40>{}); break;
    case 48: go(std::integral_constant<int, 48>{}); break;
    case 56: go(std::integral_constant<int, 56>{}); break;
    default: go(std::integral_constant<int, 64>{}); break;
  }
  return hipGetLastError();
}

hipError_t launch_blend_out(const float* I2, const ViewDesc* views, int n_img, int Hp, int Wp, int H,
                            int W, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  hipLaunchKernelGGL(blend_out_k, grid1((long)H * W, n_img), dim3(TPB), 0, s, I2, views, Hp, Wp, H, W);
  return hipGetLastError();
}

hipError_t launch_extract(const void* src, DType dt, int ld, int C, long n_pix, float* dst,
                          hipStream_t s) {
  if (n_pix <= 0) return hipSuccess;
  if (dt == DType::F32)
    hipLaunchKernelGGL(extract_k<float>, grid1(n_pix, 1), dim3(TPB), 0, s, (const float*)src, ld, C,
                       n_pix, dst);
  else
    hipLaunchKernelGGL(extract_k<bf16>, grid1(n_pix, 1), dim3(TPB), 0, s, (const bf16*)src, ld, C,
                       n_pix, dst);
  return hipGetLastError();
}

hipError_t launch_pack_nhwc(const float* src, int n_img, int C, int H, int W, void* dst, int ld,
                            DType dt, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  if (dt == DType::F32)
    hipLaunchKernelGGL(pack_nhwc_k<float>, grid1((long)H * W, n_img), dim3(TPB), 0, s, src, C, H, W,
                       (float*)dst, ld);
  else
    hipLaunchKernelGGL(pack_nhwc_k<bf16>, grid1((long)H * W, n_img), dim3(TPB), 0, s, src, C, H, W,
                       (bf16*)dst, ld);
  return hipGetLastError();
}

}  // namespace ffv
