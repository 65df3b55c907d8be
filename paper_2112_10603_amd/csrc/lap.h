// Laplacian-pyramid colour loss (section 3.1, "Loss functions", Eq. 3) and
// its gradient: device launcher and workspace size.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ffv {

constexpr int kLapLevels = 5;    // band levels of Eq. 3
constexpr int kLapMinSize = 33;  // mirror padding needs 3 samples at level 5

// Device bytes the loss of n_img images of H x W (3 channels) needs, with
// or without the gradient.
size_t lap_workspace_bytes(int n_img, int H, int W, bool grad);

// loss[i] = sum_k 2^(k-1) mean |L^k(x_i) - L^k(gt_i)| over the five band
// levels; grad (nullable) = d loss[i] / d x_i. x, gt, grad: planar
// [n_img][3][H][W] float32; loss: [n_img] float32; all device memory, as is
// the workspace of at least lap_workspace_bytes.
hipError_t launch_lap_loss(const float* x, const float* gt, int n_img, int H, int W, float* loss, float* grad,
                           void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace ffv
