// Shared body of the op-level convolution entry points (ffv_op_conv and its
// no-allocation variant).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/ffv.h"

namespace ffv {

// Device memory a call carves its buffers from (each 256-byte aligned):
// base is a device address of cap bytes.
struct OpConvScratch {
  void* base;
  size_t cap;
};

// One convolution layer as ffv_op_conv documents it. With scratch == null
// the call allocates its device buffers and frees them before returning;
// otherwise it places them in scratch and allocates no device memory,
// failing with FFV_ERR_ARG when they do not fit.
ffv_status op_conv_run(const OpConvScratch* scratch, int32_t precision, const float* x, int32_t n,
                       int32_t cin, int32_t h, int32_t w, const float* weight, const float* bias,
                       int32_t cout, int32_t stride, int32_t transposed, int32_t relu, int32_t n_tile,
                       int32_t tile_w, float* y, void* stream);

// Sets the calling thread's ffv_last_error message and returns code.
ffv_status op_fail(int code, const char* msg);

}  // namespace ffv
