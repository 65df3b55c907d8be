// ffv_op_conv_noalloc: the op-level convolution with its device buffers in
// a fixed per-device array instead of hipMalloc'd memory, for callers that
// cannot allocate.
#include <mutex>

#include <hip/hip_runtime.h>

#include "../../include/ffv.h"
#include "op_conv.h"

namespace {

// Scratch of every ffv_op_conv_noalloc call on a device: the NHWC input
// copy, packed weights, bias, NHWC output and zero block. Each device holds
// its own copy, at its own address, until the process ends.
constexpr size_t kScratchBytes = (size_t)FFV_OP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

extern "C" ffv_status ffv_op_conv_noalloc(int32_t precision, const float* x, int32_t n, int32_t cin,
                                          int32_t h, int32_t w, const float* weight, const float* bias,
                                          int32_t cout, int32_t stride, int32_t transposed, int32_t relu,
                                          int32_t n_tile, int32_t tile_w, float* y, void* stream) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return ffv::op_fail(FFV_ERR_DEVICE, "no current HIP device");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      // first call on this device (which is current): the array's device
      // address; host code never uses the array's own name
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return ffv::op_fail(FFV_ERR_DEVICE, hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    base = g_ptr[dev];
  }
  const ffv::OpConvScratch sc{base, kScratchBytes};
  return ffv::op_conv_run(&sc, precision, x, n, cin, h, w, weight, bias, cout, stride, transposed, relu,
                          n_tile, tile_w, y, stream);
}
