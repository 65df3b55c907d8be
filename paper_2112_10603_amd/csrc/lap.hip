// Laplacian-pyramid colour loss of the paper's training objective (section
// 3.1, "Loss functions", Eq. 3) and its gradient with respect to the
// synthesised image.
//
// Each level is linear in the image, so the pyramid is built on the
// difference D = x - gt: G^1 = D, G^(i+1) = even samples of blur(G^i), band
// L^i = G^i - expand(G^(i+1)), i = 1..5, with blur the separable binomial
// filter [1, 4, 6, 4, 1] / 16 under mirror padding (the edge sample is not
// repeated) and expand = blur with gain 2 per axis of the zero-inserted
// coarser level. The loss of an image is sum_i 2^(i-1) mean |L^i|. Every
// plane (image, channel) is an independent h x w array; one thread per
// output sample.
//
// Reductions: each workgroup reduces |L| of its samples in fp32 across the
// wavefront (DPP/shuffle) and the workgroup, and writes one double partial;
// a final kernel sums an image's partials in a fixed order in double, so
// the result does not depend on scheduling.
//
// Gradient: with seeds s_i = 2^(i-1) / N_i * sign(L^i) (sign 0 at 0), the
// derivative reaching G^i is a_i = s_i + R^T(a_(i+1) - E^T(s_i)), from the
// coarsest level down (a_6 = 0), where R = decimate . blur and
// E = blur_gain2 . zero-insert; the transposes gather over the taps that
// read a sample, including the mirror-folded ones.
#include <algorithm>

#include "common.h"
#include "lap.h"

namespace ffv {

namespace {

constexpr int TPB = 256;

__device__ __constant__ float kBin[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};

__device__ inline int mirror(int i, int n) {
  i = i < 0 ? -i : i;
  return i > n - 1 ? 2 * (n - 1) - i : i;
}

// Weight with which output j of the mirror-padded blur along an axis of
// length n reads input i (sum over the taps that land on i).
__device__ inline float blur_w(int j, int i, int n) {
  float w = 0.f;
#pragma unroll
  for (int t = 0; t < 5; ++t) w += mirror(j + t - 2, n) == i ? kBin[t] : 0.f;
  return w;
}

// G^(i+1) = reduce(G^i) for every plane; G^1 = a - b when b is given.
__global__ void reduce_k(const float* a, const float* b, int h, int w, int ho, int wo, float* out) {
  const long plane = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= (long)ho * wo) return;
  const int y = (int)(p / wo), x = (int)(p % wo);
  const float* pa = a + plane * h * w;
  const float* pb = b ? b + plane * h * w : nullptr;
  int xs[5];
#pragma unroll
  for (int t = 0; t < 5; ++t) xs[t] = mirror(2 * x + t - 2, w);
  float acc = 0.f;
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const long row = (long)mirror(2 * y + u - 2, h) * w;
    float r = 0.f;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const float v = pa[row + xs[t]] - (pb ? pb[row + xs[t]] : 0.f);
      r += kBin[t] * v;
    }
    acc += kBin[u] * r;
  }
  out[plane * ho * wo + p] = acc;
}

// expand(G^(i+1)) at (y, x) of an h x w level: zero-inserted samples sit at
// even mirrored positions; gain 2 per axis.
__device__ inline float expand_at(const float* g, int hn, int wn, int h, int w, int y, int x) {
  float acc = 0.f;
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int yy = mirror(y + u - 2, h);
    if (yy & 1) continue;
    float r = 0.f;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const int xx = mirror(x + t - 2, w);
      if (xx & 1) continue;
      r += kBin[t] * g[(long)(yy >> 1) * wn + (xx >> 1)];
    }
    acc += kBin[u] * r;
  }
  return 4.f * acc;
}

// Band L^i = G^i - expand(G^(i+1)) of every plane: per-workgroup partial sum
// of |L| (double), and the gradient seed weight * sign(L) when seed != null.
__global__ void band_k(const float* a, const float* b, const float* gnext, int h, int w, int hn, int wn,
                       float weight, float* seed, double* partial) {
  const long plane = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  float v = 0.f;
  if (p < (long)h * w) {
    const int y = (int)(p / w), x = (int)(p % w);
    const long o = plane * h * w + p;
    const float g = a[o] - (b ? b[o] : 0.f);
    const float l = g - expand_at(gnext + plane * hn * wn, hn, wn, h, w, y, x);
    v = fabsf(l);
    if (seed) seed[o] = l > 0.f ? weight : (l < 0.f ? -weight : 0.f);
  }
  // wavefront reduction, then the workgroup's four wavefronts
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __shared__ float wsum[TPB / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) s += (double)wsum[i];
    partial[plane * gridDim.x + blockIdx.x] = s;
  }
}

// acc[img] (+)= weight * sum of the partials of its 3 planes, in a fixed
// order; the first level assigns.
__global__ void sum_k(const double* partial, int blocks_per_plane, int n_img, double weight, int first,
                      double* acc) {
  const int img = blockIdx.x * blockDim.x + threadIdx.x;
  if (img >= n_img) return;
  double s = 0.0;
  for (long i = 0; i < 3L * blocks_per_plane; ++i) s += partial[(long)img * 3 * blocks_per_plane + i];
  acc[img] = (first ? 0.0 : acc[img]) + weight * s;
}

__global__ void finish_k(const double* acc, int n_img, float* loss) {
  const int img = blockIdx.x * blockDim.x + threadIdx.x;
  if (img < n_img) loss[img] = (float)acc[img];
}

// t = a_next - E^T(s) on the coarser level (hn x wn): E^T(s)[p][q] =
// 4 * sum over fine (j, jj) of B[j][2p] B[jj][2q] s[j][jj].
__global__ void et_k(const float* anext, const float* s, int h, int w, int hn, int wn, float* t) {
  const long plane = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= (long)hn * wn) return;
  const int y = (int)(p / wn), x = (int)(p % wn);
  const float* ps = s + plane * h * w;
  float acc = 0.f;
  for (int j = max(0, 2 * y - 4); j <= min(h - 1, 2 * y + 4); ++j) {
    const float wy = blur_w(j, 2 * y, h);
    if (wy == 0.f) continue;
    float r = 0.f;
    for (int jj = max(0, 2 * x - 4); jj <= min(w - 1, 2 * x + 4); ++jj) {
      const float wx = blur_w(jj, 2 * x, w);
      if (wx != 0.f) r += wx * ps[(long)j * w + jj];
    }
    acc += wy * r;
  }
  const long o = plane * hn * wn + p;
  t[o] = (anext ? anext[o] : 0.f) - 4.f * acc;
}

// a = s + R^T(t) on the finer level (h x w): R^T(t)[i][ii] = sum over even
// (j, jj) of B[j][i] B[jj][ii] t[j/2][jj/2].
__global__ void rt_k(const float* s, const float* t, int h, int w, int hn, int wn, float* a) {
  const long plane = blockIdx.y;
  const long p = (long)blockIdx.x * TPB + threadIdx.x;
  if (p >= (long)h * w) return;
  const int y = (int)(p / w), x = (int)(p % w);
  const float* pt = t + plane * hn * wn;
  float acc = 0.f;
  for (int j = max(0, y - 4) & ~1; j <= min(h - 1, y + 4); j += 2) {
    const float wy = blur_w(j, y, h);
    if (wy == 0.f) continue;
    float r = 0.f;
    for (int jj = max(0, x - 4) & ~1; jj <= min(w - 1, x + 4); jj += 2) {
      const float wx = blur_w(jj, x, w);
      if (wx != 0.f) r += wx * pt[(long)(j >> 1) * wn + (jj >> 1)];
    }
    acc += wy * r;
  }
  const long o = plane * h * w + p;
  a[o] = s[o] + acc;
}

inline unsigned blocks(long n) { return (unsigned)((n + TPB - 1) / TPB); }

// Level sizes (level 0 is the image) and the workspace layout: loss
// accumulators, reduction partials, levels 1..5 (reused by the backward pass
// for its per-level t and a), and the gradient seeds of levels 0..4. Each
// buffer starts on a 256-byte boundary. With base == null only the size is
// computed.
struct LapPlan {
  int h[kLapLevels + 1], w[kLapLevels + 1];
  double* acc;
  double* partial;
  float* G[kLapLevels + 1];
  float* S[kLapLevels];
  size_t bytes;
};

LapPlan lap_plan(int n_img, int H, int W, bool grad, void* base) {
  LapPlan L{};
  L.h[0] = H;
  L.w[0] = W;
  for (int i = 0; i < kLapLevels; ++i) {
    L.h[i + 1] = (L.h[i] + 1) / 2;
    L.w[i + 1] = (L.w[i] + 1) / 2;
  }
  const size_t planes = 3 * (size_t)n_img;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = base ? static_cast<char*>(base) + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return r;
  };
  L.acc = reinterpret_cast<double*>(take((size_t)n_img * 8));
  size_t max_part = 0;
  for (int i = 0; i < kLapLevels; ++i) max_part = std::max(max_part, (size_t)blocks((long)L.h[i] * L.w[i]));
  L.partial = reinterpret_cast<double*>(take(planes * max_part * 8));
  for (int i = 1; i <= kLapLevels; ++i) L.G[i] = reinterpret_cast<float*>(take(planes * L.h[i] * L.w[i] * 4));
  if (grad)
    for (int i = 0; i < kLapLevels; ++i) L.S[i] = reinterpret_cast<float*>(take(planes * L.h[i] * L.w[i] * 4));
  L.bytes = off;
  return L;
}

}  // namespace

size_t lap_workspace_bytes(int n_img, int H, int W, bool grad) { return lap_plan(n_img, H, W, grad, nullptr).bytes; }

hipError_t launch_lap_loss(const float* x, const float* gt, int n_img, int H, int W, float* loss, float* grad,
                           void* ws, size_t ws_bytes, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  if (H < kLapMinSize || W < kLapMinSize || !ws) return hipErrorInvalidValue;
  const LapPlan P = lap_plan(n_img, H, W, grad != nullptr, ws);
  if (P.bytes > ws_bytes) return hipErrorInvalidValue;
  const long planes = 3L * n_img;
  const int* hs = P.h;
  const int* wsz = P.w;
  double* acc = P.acc;
  double* partial = P.partial;
  float* const* G = P.G;
  const float* const* S = P.S;
  hipError_t e;

  // forward: reduce chain, then the bands and their sums (band i uses levels
  // i and i+1; level 0 is x - gt, read directly)
  for (int i = 0; i < kLapLevels; ++i) {
    const float* a = i == 0 ? x : G[i];
    const float* b = i == 0 ? gt : nullptr;
    hipLaunchKernelGGL(reduce_k, dim3(blocks((long)hs[i + 1] * wsz[i + 1]), (unsigned)planes), dim3(TPB), 0, s, a,
                       b, hs[i], wsz[i], hs[i + 1], wsz[i + 1], G[i + 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int i = 0; i < kLapLevels; ++i) {
    const float* a = i == 0 ? x : G[i];
    const float* b = i == 0 ? gt : nullptr;
    const long n = (long)hs[i] * wsz[i];
    const double weight = (double)(1 << i) / (3.0 * (double)n);  // 2^(i-1) / N_i, N_i = 3 h w
    const unsigned nb = blocks(n);
    hipLaunchKernelGGL(band_k, dim3(nb, (unsigned)planes), dim3(TPB), 0, s, a, b, G[i + 1], hs[i], wsz[i],
                       hs[i + 1], wsz[i + 1], (float)weight, grad ? const_cast<float*>(S[i]) : nullptr, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sum_k, dim3((unsigned)((n_img + 63) / 64)), dim3(64), 0, s, partial, (int)nb, n_img, weight,
                       i == 0 ? 1 : 0, acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finish_k, dim3((unsigned)((n_img + 63) / 64)), dim3(64), 0, s, acc, n_img, loss);
  if ((e = hipGetLastError()) != hipSuccess || !grad) return e;

  // backward, coarsest level first: t lives on level i+1, a on level i
  // (the G buffers are reused: G^(i+1) holds t, then a of level i+1 is dead)
  float* a_next = nullptr;  // a_(i+1), on level i+1
  for (int i = kLapLevels - 1; i >= 0; --i) {
    float* t = G[i + 1];  // G^(i+1) is no longer needed
    hipLaunchKernelGGL(et_k, dim3(blocks((long)hs[i + 1] * wsz[i + 1]), (unsigned)planes), dim3(TPB), 0, s, a_next,
                       S[i], hs[i], wsz[i], hs[i + 1], wsz[i + 1], t);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* a = i == 0 ? grad : G[i];
    hipLaunchKernelGGL(rt_k, dim3(blocks((long)hs[i] * wsz[i]), (unsigned)planes), dim3(TPB), 0, s, S[i], t, hs[i],
                       wsz[i], hs[i + 1], wsz[i + 1], a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    a_next = a;
  }
  return hipSuccess;
}

}  // namespace ffv
