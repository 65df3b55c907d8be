// ffv_drive: a C-ABI-only driver of libffv.so (no Python, no torch).
//
// Runs the dense-view batch (n_cams synthetic cameras at H x W, the
// n_cams - 1 adjacent pairs, n_t phases t = k/(n_t+1)) through
// ffv_interpolate `reps` times, after one plain device copy of a known
// number of bytes (a reference point for hardware memory counters). The
// input images are a smooth synthetic pattern made on the device; the
// work the library does does not depend on the pixel values.
//
// usage: ffv_drive WEIGHTS [precision=1] [H=1080] [W=1920] [n_cams=8] [n_t=16] [reps=1]
//                  [tuning_file]
// (precision 2, FP8, calibrates on the first pair at t = 1/2 before the runs)
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ffv.h"

#define CHECK_HIP(x)                                                         \
  do {                                                                       \
    hipError_t e_ = (x);                                                     \
    if (e_ != hipSuccess) {                                                  \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
      return 1;                                                              \
    }                                                                        \
  } while (0)

// 1 GiB read + 1 GiB written, 16 bytes per thread
__global__ void copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void fill_value(uint4* p, long n, unsigned v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_uint4(v, v, v, v);
}

// camera j: a smooth colour pattern shifted by 4*j pixels
__global__ void make_view(float* img, int H, int W, int j) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long)H * W) return;
  const int y = (int)(p / W), x = (int)(p % W);
  const float u = (float)(x + 4 * j), v = (float)y;
  img[p] = 0.5f + 0.4f * __sinf(0.013f * u + 0.007f * v);
  img[(long)H * W + p] = 0.5f + 0.4f * __sinf(0.011f * u - 0.009f * v + 1.0f);
  img[2L * H * W + p] = 0.5f + 0.4f * __sinf(0.017f * u + 0.005f * v + 2.0f);
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s WEIGHTS [precision] [H] [W] [n_cams] [n_t] [reps] [tuning]\n",
                 argv[0]);
    return 2;
  }
  const int precision = argc > 2 ? std::atoi(argv[2]) : 1;
  const int H = argc > 3 ? std::atoi(argv[3]) : 1080;
  const int W = argc > 4 ? std::atoi(argv[4]) : 1920;
  const int n_cams = argc > 5 ? std::atoi(argv[5]) : 8;
  const int n_t = argc > 6 ? std::atoi(argv[6]) : 16;
  const int reps = argc > 7 ? std::atoi(argv[7]) : 1;
  if (H < 2 || W < 2 || n_cams < 2 || n_t < 1 || reps < 1) return 2;

  // plain copy of a known size
  const long n16 = (1L << 30) / 16;
  uint4 *a = nullptr, *b = nullptr;
  CHECK_HIP(hipMalloc(&a, n16 * 16));
  CHECK_HIP(hipMalloc(&b, n16 * 16));
  fill_value<<<(unsigned)((n16 + 255) / 256), 256>>>(a, n16, 0x3f800000u);
  copy16<<<(unsigned)((n16 + 255) / 256), 256>>>(a, b, n16);
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipFree(a));
  CHECK_HIP(hipFree(b));
  std::printf("copy16: %ld bytes read, %ld bytes written\n", n16 * 16, n16 * 16);

  const long img = 3L * H * W;
  float* cams = nullptr;
  CHECK_HIP(hipMalloc(&cams, sizeof(float) * img * n_cams));
  for (int j = 0; j < n_cams; ++j)
    make_view<<<(unsigned)(((long)H * W + 255) / 256), 256>>>(cams + j * img, H, W, j);
  const int n_pairs = n_cams - 1;
  float* out = nullptr;
  CHECK_HIP(hipMalloc(&out, sizeof(float) * img * n_pairs * n_t));
  CHECK_HIP(hipDeviceSynchronize());

  ffv_opts o;
  ffv_default_opts(&o);
  o.precision = precision;
  o.workspace_bytes = 128ULL << 30;
  o.graphs = 0;  // eager launches: hardware counters are read per dispatch
  ffv_net* net = nullptr;
  if (ffv_create_net(argv[1], &o, &net) != FFV_OK) {
    std::fprintf(stderr, "ffv_create_net: %s\n", ffv_last_error());
    return 1;
  }
  if (argc > 8) {
    int32_t n_loaded = 0;
    if (ffv_load_tuning(net, argv[8], &n_loaded) != FFV_OK) {
      std::fprintf(stderr, "ffv_load_tuning: %s\n", ffv_last_error());
      ffv_destroy_net(net);
      return 1;
    }
    std::printf("loaded %d conv tile choices from %s\n", n_loaded, argv[8]);
  }
  if (precision == 2) {
    // FP8 nets quantise after a calibration pass: the first pair at t = 1/2
    ffv_pair cal = {cams, cams + img, H, W};
    if (ffv_calibrate(net, &cal, 0.5f) != FFV_OK) {
      std::fprintf(stderr, "ffv_calibrate: %s\n", ffv_last_error());
      ffv_destroy_net(net);
      return 1;
    }
    std::printf("calibrated on the first pair at t = 0.5\n");
  }
  std::vector<ffv_pair> pairs(n_pairs);
  for (int i = 0; i < n_pairs; ++i) pairs[i] = {cams + i * img, cams + (i + 1) * img, H, W};
  std::vector<float> ts(n_t);
  for (int k = 0; k < n_t; ++k) ts[k] = (float)(k + 1) / (float)(n_t + 1);
  for (int r = 0; r < reps; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    if (ffv_interpolate(net, pairs.data(), n_pairs, ts.data(), n_t, out) != FFV_OK) {
      std::fprintf(stderr, "ffv_interpolate: %s\n", ffv_last_error());
      ffv_destroy_net(net);
      return 1;
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::printf("rep %d: %d views of %dx%d in %.2f ms (%.1f views/s)\n", r, n_pairs * n_t, H, W, ms,
                1000.0 * n_pairs * n_t / ms);
    std::fflush(stdout);
  }
  ffv_destroy_net(net);
  CHECK_HIP(hipFree(out));
  CHECK_HIP(hipFree(cams));
  return 0;
}
