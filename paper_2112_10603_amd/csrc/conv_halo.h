// Halo-reuse variant of the implicit-GEMM convolution for layers with few
// output channels and a 3x3 neighbourhood at stride 1: 3x3 convs with
// stride 1 and phase-merged transposed convs (supplementary layer table:
// the flow/mask heads and the last decoder layers), whose input channels
// are a multiple of the K step.
//
// The generic kernel fetches a 256-pixel input window per (tap, channel
// slice) step, so every input pixel comes from L2 nine times; for these
// layers that traffic, not the MFMAs, sets the time. Here a workgroup owns
// a 16x16 block of output pixels and 32 output channels, and per channel
// slice it loads the 18x18 input halo once plus the weights of all nine
// taps; the nine taps then read shifted windows of the halo from LDS. Both
// are double-buffered: the next slice's halo and weights load while this
// slice's 9 taps x (KB/16) MFMA rounds run. The K order (slice major, taps
// inside) is the one the packed weights already use.
#pragma once

#include "conv_kernel.h"

namespace ffv {
namespace convk {

struct Halo {
  static constexpr int NT = 512;              // 8 waves
  static constexpr int TW = 16, TH = 16;      // output block
  static constexpr int HW = TW + 2, HH = TH + 2;
  static constexpr int NH = HW * HH;          // halo pixels
  static constexpr int BN = 32;               // output channels (GEMM rows) per block
  static constexpr int KB = 128;              // bytes of a pixel's channel slice
  static constexpr int CH = KB / 16;          // 16-byte chunks per row
  static constexpr int A_VECS = NH * CH;
  static constexpr int B_VECS = 9 * BN * CH;
  static constexpr int A_IT = (A_VECS + NT - 1) / NT;
  static constexpr int B_IT = (B_VECS + NT - 1) / NT;
  // 16 consecutive rows cover distinct 16-byte bank groups of a 256-byte window
  __device__ static inline int key(int row) { return (row >> 1) & (CH - 1); }
  __device__ static inline int swz(int row, int chunk) { return row * CH + (chunk ^ key(row)); }
};

template <typename T>
__global__ __launch_bounds__(Halo::NT) void conv_halo(ConvArgs a) {
  using H = Halo;
  constexpr int NT = H::NT, CH = H::CH, TW = H::TW, HW = H::HW, BN = H::BN;
  constexpr int BK = H::KB / (int)sizeof(T), VEC = 16 / (int)sizeof(T);
  constexpr int A_IT = H::A_IT, B_IT = H::B_IT, A_VECS = H::A_VECS, B_VECS = H::B_VECS;

  __shared__ __attribute__((aligned(16))) uint4 Ah[2][H::NH * CH];
  __shared__ __attribute__((aligned(16))) uint4 Bh[2][9 * BN * CH];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lrow = lane & 31, lhalf = lane >> 5;
  const int merged = a.transposed == 2;

  // XCD-aware M-tile order, as in the generic kernel
  const int gx = gridDim.x, bx = blockIdx.x;
  const int xcd = bx & 7, q = gx >> 3, r = gx & 7;
  const int mt = xcd * q + min(xcd, r) + (bx >> 3);
  const int tiles_x = (a.Wo + TW - 1) / TW, tiles_y = (a.Ho + H::TH - 1) / H::TH;
  const int img_t = mt / (tiles_x * tiles_y);
  const int rem_t = mt - img_t * tiles_x * tiles_y;
  const int ty0 = (rem_t / tiles_x) * H::TH, tx0 = (rem_t % tiles_x) * TW;
  const int n0 = blockIdx.y * BN;
  const int chunk = tid % CH;

  const T* in = reinterpret_cast<const T*>(a.in) + (long)img_t * a.in_img_stride;
  const T* wgt = reinterpret_cast<const T*>(a.wgt);
  const T* zero = reinterpret_cast<const T*>(a.zero);

  // halo loads: slot v = tid + i*NT holds (halo pixel v / CH, physical chunk)
  int h_off[A_IT];
  bool h_ok[A_IT];
#pragma unroll
  for (int i = 0; i < A_IT; ++i) {
    const int v = tid + i * NT;
    const int hrow = v / CH;
    const int iy = ty0 - 1 + hrow / HW, ix = tx0 - 1 + hrow % HW;
    h_ok[i] = v < A_VECS && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
    h_off[i] = h_ok[i] ? (iy * a.Wi + ix) * a.in_ld + (chunk ^ H::key(hrow)) * VEC : 0;
  }
  // weight loads: slot v holds (tap, row n) = ((v / CH) / BN, (v / CH) % BN)
  const T* b_src[B_IT];
#pragma unroll
  for (int i = 0; i < B_IT; ++i) {
    const int v = tid + i * NT;
    const int brow = v < B_VECS ? v / CH : 0;
    const int tap = brow / BN, n = brow - tap * BN;
    b_src[i] = wgt + (long)(n0 + n) * a.K_pad + tap * BK + (chunk ^ H::key(brow)) * VEC;
  }
  const int n_slices = a.cin_pad / BK;

  auto issue = [&](int s, int buf) {
    const int c_s = s * BK;
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const T* src = h_ok[i] ? in + h_off[i] + c_s : zero;
      if (A_VECS % NT == 0 || tid + i * NT < A_VECS) load_to_lds(src, &Ah[buf][i * NT + wave * 64]);
    }
#pragma unroll
    for (int i = 0; i < B_IT; ++i) {
      const T* src = b_src[i] + (long)s * 9 * BK;
      if (B_VECS % NT == 0 || tid + i * NT < B_VECS) load_to_lds(src, &Bh[buf][i * NT + wave * 64]);
    }
  };

  // this lane's output pixel (GEMM row) in the 16x16 block, for A fragments
  const int prow = wave * 32 + lrow;
  const int py = prow / TW, pxx = prow % TW;
  f32x16 acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;

  auto compute = [&](int buf) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int hidx = (py + tap / 3) * HW + pxx + tap % 3;  // (y + dy + 1, x + dx + 1)
      const int brow = tap * BN + lrow;
      if constexpr (sizeof(T) == 1) {
#pragma unroll
        for (int s = 0; s < CH / 4; ++s) {
          const int ch = lhalf * (CH / 2) + 2 * s;
          mfma_f8(acc, Ah[buf][H::swz(hidx, ch)], Ah[buf][H::swz(hidx, ch + 1)],
                  Bh[buf][H::swz(brow, ch)], Bh[buf][H::swz(brow, ch + 1)]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < CH / 2; ++s) {
          const int ch = lhalf * (CH / 2) + s;
          mfma_chunk<T>(acc, Ah[buf][H::swz(hidx, ch)], Bh[buf][H::swz(brow, ch)]);
        }
      }
    }
  };

  constexpr int LPS = A_IT + B_IT;
  (void)LPS;
  if (n_slices > 0) issue(0, 0);
  for (int s = 0; s < n_slices; ++s) {
    wait_vm<0>();
    __syncthreads();
    if (s + 1 < n_slices) issue(s + 1, (s + 1) & 1);
    compute(s & 1);
  }

  // Epilogue (pixels as A): lane l holds channel n0 + l%32 for 16 pixels.
  const int cout_m = merged ? a.cout : 1;
  const int n = n0 + lrow;
  long col = 0;
  int o = 0;
  bool n_ok;
  if (!merged) {
    n_ok = n < a.cout;
    o = n;
    col = n;
  } else {
    n_ok = n < 4 * cout_m;
    const int ph = n_ok ? n / cout_m : 0;
    o = n - ph * cout_m;
    col = ((long)(ph >> 1) * a.Wout + (ph & 1)) * a.out_ld + o;
  }
  if (!n_ok) return;
  const float bn = a.bias[o];
  const float ws = a.w_scale ? a.w_scale[o] : 1.f;
  float amax = 0.f;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = wave * 32 + (e >> 2) * 8 + lhalf * 4 + (e & 3);
    int oy = ty0 + row / TW, ox = tx0 + row % TW;
    if (oy >= a.Ho || ox >= a.Wo) continue;
    if (a.transposed) {  // phase-merged: the GEMM grid point's phase-(0, 0) output
      oy *= 2;
      ox *= 2;
    }
    float v = acc[e] * ws + bn;
    if (a.relu) v = fmaxf(v, 0.f);
    amax = fmaxf(amax, fabsf(v));
    store_out<T>(a, (long)img_t * a.out_img_stride + ((long)oy * a.Wout + ox) * a.out_ld + col, o, v);
  }
  if (a.amax) atomicMax(reinterpret_cast<unsigned*>(a.amax) + o, __float_as_uint(amax));
}

// Whether the halo kernel covers the launch.
inline bool halo_ok(const ConvArgs& a, int bk) {
  const bool s1 = (a.transposed == 0 && a.stride == 1) || a.transposed == 2;
  return s1 && a.taps == 9 && a.cin_pad % bk == 0 && a.K_pad == 9 * a.cin_pad && a.tile_w == Halo::TW &&
         a.Hi == a.Ho && a.Wi == a.Wo;
}

template <typename T>
hipError_t launch_halo(const ConvArgs& a, hipStream_t s) {
  constexpr int BK = Halo::KB / (int)sizeof(T), VEC = 16 / (int)sizeof(T);
  const int n_tiles = (a.n_rows + Halo::BN - 1) / Halo::BN;
  if (!halo_ok(a, BK) || a.n_rows <= 0 || n_tiles * Halo::BN > a.cout_pad || a.in_ld % VEC != 0)
    return hipErrorInvalidValue;
  if ((long)a.Hi * a.Wi * a.in_ld >= (1L << 31)) return hipErrorInvalidValue;
  const long tiles = (long)a.n_img * ((a.Ho + Halo::TH - 1) / Halo::TH) * ((a.Wo + Halo::TW - 1) / Halo::TW);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(conv_halo<T>, dim3((unsigned)tiles, (unsigned)n_tiles, 1), dim3(Halo::NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace convk
}  // namespace ffv
