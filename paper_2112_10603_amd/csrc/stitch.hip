// Multi-view cluster frame (the paper's Multiview Organizer, section 3.2,
// and the supplement's 16-views-per-side clusters): a camera's real view at
// full resolution between two blocks of its neighbouring views, each
// downscaled by g in both directions (g x g box mean) and tiled g x g in
// raster order, so a side's g*g views fill exactly one H x W block:
//   frame [3][H][3W] = [left block | real view | right block].
// Memory-bound: one thread per output pixel; a tile pixel reads a g x g
// block of its source view (rows of g consecutive floats: one 16-byte load
// per row when g = 4), consecutive threads take consecutive output pixels.
#include "common.h"

namespace ffv {

namespace {

constexpr int TPB = 256;

template <int G>
__global__ void stitch_k(StitchArgs a) {
  const long HW3 = 3L * a.H * a.W;  // pixels of one output plane
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= HW3) return;
  const int W3 = 3 * a.W;
  const int y = (int)(p / W3), x = (int)(p % W3);
  const int block = x / a.W, xl = x - block * a.W;
  const long HWs = (long)a.H * a.W;
  float v[3];
  if (block == 1) {
    const long q = (long)y * a.W + xl;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = a.hr[c * HWs + q];
  } else {
    const int th = a.H / G, tw = a.W / G;
    const int r = y / th, qd = xl / tw;
    const float* src = a.views[(block == 0 ? 0 : a.n) + r * G + qd];
    const int sy = G * (y - r * th), sx = G * (xl - qd * tw);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* s = src + c * HWs + (long)sy * a.W + sx;
      float acc = 0.f;
#pragma unroll
      for (int i = 0; i < G; ++i) {
        if constexpr (G == 4) {
          const float4 t = *reinterpret_cast<const float4*>(s + (long)i * a.W);
          acc += (t.x + t.y) + (t.z + t.w);
        } else {
#pragma unroll
          for (int j = 0; j < G; ++j) acc += s[(long)i * a.W + j];
        }
      }
      v[c] = acc * (1.f / (G * G));
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.out[c * HW3 + p] = v[c];
}

}  // namespace

hipError_t launch_stitch(const StitchArgs& a, hipStream_t s) {
  const long n = 3L * a.H * a.W;
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + TPB - 1) / TPB));
  switch (a.g) {
    case 1: hipLaunchKernelGGL(stitch_k<1>, grid, dim3(TPB), 0, s, a); break;
    case 2: hipLaunchKernelGGL(stitch_k<2>, grid, dim3(TPB), 0, s, a); break;
    case 4: hipLaunchKernelGGL(stitch_k<4>, grid, dim3(TPB), 0, s, a); break;
    case 8: hipLaunchKernelGGL(stitch_k<8>, grid, dim3(TPB), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ffv
