// Implicit-GEMM convolution on CDNA4 matrix cores (gfx950).
//
// Covers every convolution of the network (supplementary layer table):
// 3x3 convs with padding 1 and stride 1 or 2, and 4x4 stride-2 padding-1
// transposed convs, which split into four output phases, each a 2x2-tap
// conv over the input grid (blockIdx.z selects the phase).
//
// GEMM view: M = output pixels (images folded in), N = output channels,
// K = (tap, input channel). A workgroup of 4 waves computes a BM x BN tile;
// each wave owns a (BM/WM) x (BN/WN) block of 32x32 MFMA fragments. Per K
// step of 32 the A tile (gathered from NHWC activations, zero outside the
// image) and the B tile (packed weights, K contiguous) are staged in LDS with
// a register prefetch of the next step.
//
// Inside a 32-wide K step, lane half h = lane/32 owns k in [16h, 16h+16);
// the MFMA's k positions are fed in that order for both operands, so the
// sum over k is the full dot product whatever the instruction's internal k
// order. Accumulation is fp32 in every precision.
#include "common.h"

namespace ffv {

namespace {

constexpr int BK = 32;
constexpr int VEC = 8;  // elements per gathered vector (8 channels of one tap)
constexpr int KV = BK / VEC;
constexpr int NTHREADS = 256;

template <typename T>
struct Vec8 {
  uint4 v[sizeof(T) * VEC / 16];
};

template <typename T>
__device__ inline Vec8<T> load_vec(const T* p) {
  Vec8<T> r;
  const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) * VEC / 16); ++i) r.v[i] = q[i];
  return r;
}

template <typename T>
__device__ inline Vec8<T> zero_vec() {
  Vec8<T> r;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) * VEC / 16); ++i) r.v[i] = make_uint4(0, 0, 0, 0);
  return r;
}

template <typename T>
__device__ inline void store_vec(T* p, const Vec8<T>& r) {
  uint4* q = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) * VEC / 16); ++i) q[i] = r.v[i];
}

// Per-lane operand fragment for one 32-wide K step: 16 consecutive k values.
template <typename T>
struct Frag {
  T e[16];
};

template <typename T>
__device__ inline void mfma_step(f32x16& acc, const Frag<T>& a, const Frag<T>& b);

template <>
__device__ inline void mfma_step<float>(f32x16& acc, const Frag<float>& a, const Frag<float>& b) {
#pragma unroll
  for (int s = 0; s < 16; ++s)
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.e[s], b.e[s], acc, 0, 0, 0);
}

template <>
__device__ inline void mfma_step<bf16>(f32x16& acc, const Frag<bf16>& a, const Frag<bf16>& b) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bf16x8 av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      av[i] = a.e[s * 8 + i];
      bv[i] = b.e[s * 8 + i];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
}

template <typename T>
__device__ inline void store_out(const ConvArgs& a, long off, float v);

template <typename T, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(NTHREADS) void conv_igemm(ConvArgs a) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  static_assert(FM >= 1 && FN >= 1, "wave tile >= 32x32");
  constexpr int PADK = 16 / (int)sizeof(T);  // one 16-byte pad per LDS row
  constexpr int LDK = BK + PADK;
  constexpr int A_VECS = BM * KV, B_VECS = BN * KV;
  constexpr int A_IT = (A_VECS + NTHREADS - 1) / NTHREADS;
  constexpr int B_IT = (B_VECS + NTHREADS - 1) / NTHREADS;

  __shared__ __attribute__((aligned(16))) T As[BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int phase = blockIdx.z;
  const int py = phase >> 1, px = phase & 1;
  const long M = (long)a.n_img * a.Ho * a.Wo;
  const long m0 = (long)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int kv = tid % KV;

  const T* in = reinterpret_cast<const T*>(a.in);
  const T* wgt = reinterpret_cast<const T*>(a.wgt) + (long)phase * a.cout_pad * a.K_pad;

  // Rows of the A tile this thread gathers: fixed across the K loop.
  const T* a_base[A_IT];
  int a_iy[A_IT], a_ix[A_IT];
  bool a_ok[A_IT];
#pragma unroll
  for (int i = 0; i < A_IT; ++i) {
    const int v = tid + i * NTHREADS;
    const int row = v / KV;
    const long m = m0 + row;
    a_ok[i] = (v < A_VECS) && (m < M);
    const long mm = a_ok[i] ? m : 0;
    const long hw = (long)a.Ho * a.Wo;
    const long img = mm / hw;
    const int rem = (int)(mm - img * hw);
    const int oy = rem / a.Wo, ox = rem - (rem / a.Wo) * a.Wo;
    a_base[i] = in + img * a.in_img_stride;
    a_iy[i] = oy * a.stride;
    a_ix[i] = ox * a.stride;
  }

  Vec8<T> ra[A_IT], rb[B_IT];

  auto gather = [&](int kc) {
    const int k0 = kc * BK + kv * VEC;
    int dy = 0, dx = 0, c = 0;
    const bool kin = k0 < a.K;
    if (kin) {
      const int tap = k0 / a.cin_pad;
      c = k0 - tap * a.cin_pad;
      if (a.transposed) {
        dy = py - (tap >> 1);
        dx = px - (tap & 1);
      } else {
        dy = tap / 3 - 1;
        dx = tap % 3 - 1;
      }
    }
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const int iy = a_iy[i] + dy, ix = a_ix[i] + dx;
      if (kin && a_ok[i] && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi)
        ra[i] = load_vec<T>(a_base[i] + ((long)iy * a.Wi + ix) * a.in_ld + c);
      else
        ra[i] = zero_vec<T>();
    }
#pragma unroll
    for (int i = 0; i < B_IT; ++i) {
      const int v = tid + i * NTHREADS;
      if (v < B_VECS) {
        const int row = v / KV;
        const int n = n0 + row;
        if (n < a.cout_pad)
          rb[i] = load_vec<T>(wgt + (long)n * a.K_pad + kc * BK + kv * VEC);
        else
          rb[i] = zero_vec<T>();
      }
    }
  };

  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const int v = tid + i * NTHREADS;
      if (v < A_VECS) store_vec<T>(&As[(v / KV) * LDK + kv * VEC], ra[i]);
    }
#pragma unroll
    for (int i = 0; i < B_IT; ++i) {
      const int v = tid + i * NTHREADS;
      if (v < B_VECS) store_vec<T>(&Bs[(v / KV) * LDK + kv * VEC], rb[i]);
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int nk = a.K_pad / BK;
  const int lrow = lane & 31;
  const int khalf = (lane >> 5) * 16;

  gather(0);
  for (int kc = 0; kc < nk; ++kc) {
    __syncthreads();
    stash();
    __syncthreads();
    if (kc + 1 < nk) gather(kc + 1);

    Frag<T> fa[FM], fb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const T* p = &As[(wm * TM + i * 32 + lrow) * LDK + khalf];
#pragma unroll
      for (int e = 0; e < 16; ++e) fa[i].e[e] = p[e];
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const T* p = &Bs[(wn * TN + j * 32 + lrow) * LDK + khalf];
#pragma unroll
      for (int e = 0; e < 16; ++e) fb[j].e[e] = p[e];
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) mfma_step<T>(acc[i][j], fa[i], fb[j]);
  }

  // Epilogue: bias, ReLU, optional accumulate, store (NHWC, channel slice).
  const int lhalf = lane >> 5;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    long off_row[16];
    bool row_ok[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm * TM + i * 32 + (r >> 2) * 8 + lhalf * 4 + (r & 3);
      const long m = m0 + row;
      row_ok[r] = m < M;
      const long mm = row_ok[r] ? m : 0;
      const long hw = (long)a.Ho * a.Wo;
      const long img = mm / hw;
      const int rem = (int)(mm - img * hw);
      int oy = rem / a.Wo, ox = rem - (rem / a.Wo) * a.Wo;
      if (a.transposed) {
        oy = 2 * oy + py;
        ox = 2 * ox + px;
      }
      off_row[r] = img * a.out_img_stride + ((long)oy * a.Wout + ox) * a.out_ld;
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn * TN + j * 32 + lrow;
      if (n >= a.cout) continue;
      const float bn = a.bias[n];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (!row_ok[r]) continue;
        float v = acc[i][j][r] + bn;
        if (a.relu) v = fmaxf(v, 0.f);
        store_out<T>(a, off_row[r] + n, v);
      }
    }
  }
}

template <typename T>
__device__ inline void store_out(const ConvArgs& a, long off, float v) {
  if (a.out_f32) {
    float* o = reinterpret_cast<float*>(a.out) + off;
    if (a.accumulate) v += *o;
    *o = v;
  } else {
    reinterpret_cast<T*>(a.out)[off] = (T)v;
  }
}

template <typename T>
hipError_t launch_t(ConvTile tile, const ConvArgs& a, hipStream_t s) {
  const long M = (long)a.n_img * a.Ho * a.Wo;
  const int phases = a.transposed ? 4 : 1;
  int bm = 128, bn = 128;
  if (tile == ConvTile::M128_N64) bn = 64;
  if (tile == ConvTile::M128_N32) bn = 32;
  if (a.K_pad % BK != 0 || a.cin_pad % VEC != 0 || a.cout_pad % bn != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((M + bm - 1) / bm), (unsigned)(a.cout_pad / bn), phases);
  switch (tile) {
    case ConvTile::M128_N128:
      hipLaunchKernelGGL((conv_igemm<T, 128, 128, 2, 2>), grid, dim3(NTHREADS), 0, s, a);
      break;
    case ConvTile::M128_N64:
      hipLaunchKernelGGL((conv_igemm<T, 128, 64, 4, 1>), grid, dim3(NTHREADS), 0, s, a);
      break;
    case ConvTile::M128_N32:
      hipLaunchKernelGGL((conv_igemm<T, 128, 32, 4, 1>), grid, dim3(NTHREADS), 0, s, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_conv(DType dt, ConvTile tile, const ConvArgs& a, hipStream_t s) {
  if (a.n_img <= 0 || a.Ho <= 0 || a.Wo <= 0) return hipSuccess;
  if (dt == DType::F32) return launch_t<float>(tile, a, s);
  return launch_t<bf16>(tile, a, s);
}

}  // namespace ffv
