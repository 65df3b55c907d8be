// Shared declarations of the HIP library: element types, kernel argument
// structs and the host-side launchers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ffv {

typedef __bf16 bf16;
// fp8 e4m3 (OCP: bias 7, max 448, no infinities) as stored bytes
struct f8 {
  uint8_t v;
};
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float float2v;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) int i32x8;

enum class DType : int { F32 = 0, BF16 = 1, FP8 = 2 };

inline size_t dtype_size(DType t) { return t == DType::F32 ? 4 : (t == DType::BF16 ? 2 : 1); }

// One implicit-GEMM convolution launch: C[m][n] = sum_k A[m][k] * B[n][k].
//   m: output pixel of the GEMM grid (image, oy, ox), M = n_img * Ho * Wo
//   n: output channel
//   k: (tap, input channel); taps are the 9 offsets of a 3x3 conv, or the 4
//      taps of one output phase of a 4x4 stride-2 transposed conv
// Activations are NHWC with a pixel stride (ld) that may exceed the channel
// count, so a layer can read or write a channel slice of a wider buffer.
struct ConvArgs {
  const void* in;       // input base, already offset to the first channel
  long in_img_stride;   // elements between images
  int in_ld;            // elements between pixels
  int Hi, Wi;           // input size
  const void* wgt;      // packed weights [phase][Cout_pad][K_pad], act dtype
  const float* bias;    // [Cout]
  void* out;            // output base, already offset to the first channel
  long out_img_stride;
  int out_ld;
  int Ho, Wo;           // GEMM grid size (transposed: = input size)
  int Hout, Wout;       // output image size (transposed: 2x the grid)
  int cin_pad;          // input channels, multiple of 8 (zero weights past the real count)
  int K;                // taps * cin_pad
  int K_pad;            // K rounded up to the K tile
  int cout;             // real output channels
  int cout_pad;         // rows per phase in the packed weights (a multiple of 256)
  int n_rows;           // GEMM N: cout, or 4 * cout phase-merged; grid y = ceil(n_rows / BN)
  int n_img;
  int stride;           // 1 or 2 (conv); 1 for transposed
  int transposed;       // 0: 3x3 conv; 1: 4x4 s2 transposed, one output phase per
                        // blockIdx.z; 2: 4x4 s2 transposed, phase-merged (n = phase*cout + o)
  int relu;
  int out_f32;          // 1: float output, 0: activation dtype (or fp8, see out_scale)
  int accumulate;       // 1: add into the existing float output
  const float* w_scale;   // per output channel, multiplies the accumulator (fp8 weights); or null
  const float* out_scale; // per output channel: store fp8(value * out_scale[o]); or null
  float* amax;            // per output channel max |value| (calibration); or null
  int taps;             // taps in K (9, or 4 for one transposed phase)
  int tile_w;           // width of the 2-D pixel block of an M tile (divides the M tile)
  const void* zero;     // >= 16 bytes of zeros (read for taps outside the image)
};

// One launch of the implicit-GEMM kernel over up to kMax groups of images
// of different sizes (views of several resolutions in one batch): group g
// owns the workgroups first[g] .. first[g+1]-1 along grid x and runs with
// a[g]; the groups share the layer (weights, channels, mode), so grid y and
// z are common.
struct ConvGroup {
  static constexpr int kMax = 4;
  ConvArgs a[kMax];
  int n;
  int first[kMax + 1];
};

// N-tile widths the conv kernel is instantiated for (the M tile is 256);
// H32: the halo-reuse kernel (16x16 output pixels x 32 channels, stride-1
// 3x3 neighbourhoods only; the M-tile width must be 16); H256, H128: the
// conv kernel's halo variant with 256/128-channel N tiles (stride-1 3x3
// neighbourhoods and per-phase transposed convs; M-tile width 8, 16 or 32);
// R32, R64: the persistent halo kernel with the layer's weights resident in
// LDS (stride-1 3x3 neighbourhoods with at most 32/64 GEMM columns and small
// weights; M-tile width 16); S32, S64, S128: the persistent few-channel
// kernel (stride 2 or 1, 8 to 32 input channels), weights resident (M-tile
// width 16); Q256: the 256-column halo tile with its waves as 2 x 4 (on a
// per-phase transposed conv with at most 64 outputs, all four phases in one
// workgroup); P256: the H256 tile with its eight waves in two groups whose
// MFMA and memory phases alternate (same results bit for bit).
enum class ConvTile : int {
  N256 = 0, N128 = 1, N64 = 2, N32 = 3, H32 = 4, H256 = 5, H128 = 6, R32 = 7, R64 = 8, S32 = 9, S64 = 10, S128 = 11,
  Q256 = 12, P256 = 13
};
// N tile (output channels per workgroup) of a tile kind.
inline int conv_tile_bn(ConvTile t) {
  switch (t) {
    case ConvTile::N256: case ConvTile::H256: case ConvTile::Q256: case ConvTile::P256: return 256;
    case ConvTile::N128: case ConvTile::H128: case ConvTile::S128: return 128;
    case ConvTile::N64: case ConvTile::R64: case ConvTile::S64: return 64;
    default: return 32;
  }
}
// Whether the halo-reuse kernel can run a launch (tile_w is not checked).
bool conv_halo_ok(DType dt, const ConvArgs& a);
// Whether the H256/H128 halo variant can run a launch (tile_w checked).
bool conv_halo_tile_ok(DType dt, const ConvArgs& a);
// Whether the resident-weight kernel with a bn-channel N tile (32 or 64) can
// run a launch (tile_w is not checked: the kernel's block is 16 x 16).
bool conv_resident_ok(DType dt, const ConvArgs& a, int bn);
// Whether the stride-2 resident kernel with a bn-channel N tile (32, 64 or
// 128) can run a launch.
bool conv_resident_s2_ok(DType dt, const ConvArgs& a, int bn);

hipError_t launch_conv(DType dt, ConvTile tile, const ConvArgs& a, hipStream_t s);
// One launch over n (1 .. ConvGroup::kMax) groups of images of the same
// layer; with more than one group only the generic tiles (N*) and the
// two-group halo tile (P256) run it.
hipError_t launch_conv_grouped(DType dt, ConvTile tile, const ConvArgs* a, int n, hipStream_t s);
// Whether a tile can run a launch of several groups.
inline bool conv_tile_groupable(ConvTile t) {
  return t == ConvTile::N256 || t == ConvTile::N128 || t == ConvTile::N64 || t == ConvTile::N32 ||
         t == ConvTile::P256;
}
// Width of the 2-D pixel block of a 256-pixel M tile for a Ho x Wo grid:
// the least padded area, the squarest block on ties.
int conv_tile_width(int Ho, int Wo);
// K elements per pipeline step of the conv kernel for a dtype.
int conv_k_step(DType dt);

// Per-camera data on the device (all NHWC), shared by every view of the
// camera: padded image (4 floats per pixel), its quarter- and half-size
// copies, and the four context-feature levels (activation dtype).
struct CamDev {
  const float* X4;
  const float* L0;
  const float* L1;
  const void* ctx[4];
};

// Per-view description: the two cameras (indices into the CamDev table),
// the phase, where the view's planar [3][H][W] output goes, and the view's
// own size: real (h, w) and padded to multiples of 16 (hp, wp). A launch
// over views of several sizes is sized for the largest: per-view buffers
// are strided by the launch's size, each view's data laid out with its own
// width at the start of its slot, and threads past a view's own size exit.
struct ViewDesc {
  int cam_l, cam_r;
  float t;
  int hp;
  float* out;
  int wp, h, w, pad;
};

hipError_t launch_ingest(const float* const* src, int n_cam, int H, int W, int Hp, int Wp,
                         float* X4, void* Xa, DType dt, hipStream_t s);
hipError_t launch_resample4(const float* in, int n_img, int Hi, int Wi, float* out, int Ho, int Wo,
                            hipStream_t s);
hipError_t launch_assemble0(const ViewDesc* views, int n_views, const CamDev* cams, int h, int w,
                            void* x, int ld, DType dt, int t_plane, hipStream_t s);
hipError_t launch_transition(const ViewDesc* views, int n_views, const CamDev* cams, int level,
                             const float* FMprev, int hp, int wp, int h, int w, void* x, int ld,
                             float* FM, DType dt, int t_plane, hipStream_t s);
hipError_t launch_final(const ViewDesc* views, int n_views, const CamDev* cams, const float* FM,
                        int h, int w, float* I2, void* x0u, int ld, DType dt, hipStream_t s);
// Flow pyramid level k+1 from level k (k = 0: full resolution) of every
// view: in/out strided by the launch's level sizes h x w and h/2 x w/2.
hipError_t launch_flow_down(const float* in, int in_ld, const ViewDesc* views, int n_img, int k, int h, int w,
                            float* out, hipStream_t s);
hipError_t launch_ctx_warp(const ViewDesc* views, int n_views, const CamDev* cams, int level, int C,
                           const float* flow, int h, int w, void* dst, int dst_ld,
                           long dst_img_stride, DType dt, hipStream_t s);
// Multi-view cluster frame: [left block | real view | right block], each
// side g*g views box-downscaled by g and tiled in raster order.
struct StitchArgs {
  const float* hr;          // planar [3][H][W]
  const float* views[128];  // left side 0 .. n-1, right side n .. 2n-1
  int n, g, H, W;           // n = g*g views per side
  float* out;               // planar [3][H][3W]
};
hipError_t launch_stitch(const StitchArgs& a, hipStream_t s);

// Blend-only output: I2 (padded NHWC, 4 floats) cropped to planar [3][H][W]
// at each view's out pointer.
hipError_t launch_blend_out(const float* I2, const ViewDesc* views, int n_img, int Hp, int Wp, int H,
                            int W, hipStream_t s);
hipError_t launch_head(const void* u4, int ld, int C, const float* w, const float* b,
                       const float* I2, const ViewDesc* views, int n_img, int Hp, int Wp, int H,
                       int W, DType dt, hipStream_t s);
hipError_t launch_extract(const void* src, DType dt, int ld, int C, long n_pix, float* dst,
                          hipStream_t s);
hipError_t launch_pack_nhwc(const float* src, int n_img, int C, int H, int W, void* dst, int ld,
                            DType dt, hipStream_t s);

}  // namespace ffv
