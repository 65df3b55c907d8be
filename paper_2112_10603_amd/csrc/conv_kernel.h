// Implicit-GEMM convolution kernel template for CDNA4 matrix cores (gfx950).
//
// Covers every convolution of the network (supplementary layer table):
// 3x3 convs with padding 1 and stride 1 or 2, and 4x4 stride-2 padding-1
// transposed convs. A transposed conv runs either per output phase (four
// 2x2-tap convs over the input grid, blockIdx.z = phase) or, when it has few
// output channels, phase-merged: one 3x3-neighbourhood conv over the input
// grid whose N dimension holds (phase, channel), so the input tile is read
// once for all four phases.
//
// GEMM view: M = output pixels (images folded in), N = output channels,
// K = (tap, input channel). The BM pixels of an M tile form a 2-D block of
// the grid (BM / tile_w rows of tile_w pixels), so the input rows its 3x3
// taps read are shared by the block's own rows and stay in cache. A
// workgroup of WM x WN waves computes a BM x BN tile; each wave owns a block of 32x32 MFMA fragments. Each K step covers
// KB bytes of every A and B row: the A tile is gathered from NHWC
// activations, the B tile read from packed weights (K contiguous). Both go
// straight from global memory into LDS with global_load_lds_dwordx4 (no
// register staging): a lane's load lands in the 16-byte LDS slot given by
// its position in the workgroup, so each lane fetches the chunk that the
// XOR swizzle (chunk ^ f(row)) places in that slot, and taps outside the
// image read from a zero buffer. STAGES LDS buffers form a ring: the loads
// of the next STAGES - 1 steps are in flight while step k computes; one
// barrier per step. Tiles along M are assigned so that each XCD works on a contiguous
// range of output rows (its L2 keeps the shared input rows).
//
// Inside a K step, lane half h = lane/32 owns one half of the step's k
// range; the MFMA's k positions are fed in that order for both operands, so
// the sum over k is the full dot product whatever the instruction's internal
// k order. Accumulation is fp32 in every precision. Tiles with 128 or 256
// output channels in bf16/fp8 feed the weights as the MFMA's A operand, so
// a lane ends with consecutive output channels of one pixel; their
// epilogue stages the output tile through LDS and writes 16-byte chunks.
//
// HALO variant (3x3 stride-1 convs, per-phase and phase-merged transposed
// convs, whose channels are a multiple of the K step): the M tile's input
// halo ((TH + 2) x (TW + 2) pixels of one channel slice) is loaded into LDS
// once per slice, and every tap of the slice reads its shifted window of
// it, so the A bytes per slice drop from taps x BM rows to the halo's rows.
// The next slice's halo is loaded in pieces, one share per tap step of the
// current slice, into the second halo buffer; the weight tiles keep the
// two-stage ring of the generic kernel. A 256-column HALO tile over a
// per-phase transposed conv computes WN output phases at once (WN column
// groups of waves): with 2, phases (py, 0) and (py, 1) for at most 128
// outputs; with 4, all four for at most 64. The phases read the same halo
// (their 2x2 taps differ only in offset), each column group takes one
// phase, and the B tile stacks the phases' weight rows, so a K step does a
// full 256-column step's work without extra MFMAs.
#pragma once

#include <type_traits>

#include "common.h"


namespace ffv {
namespace convk {

template <typename T>
__device__ inline void mfma_chunk(f32x16& acc, const uint4& a, const uint4& b);

// 16 bytes = 8 bf16 k-values per lane: one 32x32x16 MFMA.
template <>
__device__ inline void mfma_chunk<bf16>(f32x16& acc, const uint4& a, const uint4& b) {
  bf16x8 av = __builtin_bit_cast(bf16x8, a);
  bf16x8 bv = __builtin_bit_cast(bf16x8, b);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
}

// 16 bytes = 4 fp32 k-values per lane: four 32x32x2 MFMAs.
template <>
__device__ inline void mfma_chunk<float>(f32x16& acc, const uint4& a, const uint4& b) {
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
}

typedef __attribute__((address_space(3))) void* lptr_t;

// 16 bytes from global memory straight into LDS: lane l of the wave writes
// dst_wave_base + 16*l (global_load_lds_dwordx4, M0 = LDS base). Issued as
// inline asm so the compiler does not serialise it against the operand
// reads of the other ring stage; the caller waits on vmcnt before the
// barrier that publishes the stage. M0 is saved and restored around the
// load, so its value is unchanged for the surrounding compiled code.
__device__ inline void load_to_lds(const void* src, void* dst_wave_base) {
  const uint32_t lds = __builtin_amdgcn_readfirstlane((uint32_t)(size_t)(lptr_t)dst_wave_base);
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds), "v"(src)
      : "memory");
}

// The same with a wave-uniform 64-bit base (scalar registers) and a 32-bit
// per-lane byte offset: lane l reads sbase + voff and writes
// dst_wave_base + 16*l. One offset register per lane serves every load
// whose address differs only by a uniform amount.
__device__ inline void load_to_lds_s(const void* sbase, uint32_t voff, void* dst_wave_base) {
  const uint32_t lds = __builtin_amdgcn_readfirstlane((uint32_t)(size_t)(lptr_t)dst_wave_base);
  // (readfirstlane returns a signed int: each half is widened as unsigned)
  const uint64_t b = (uint64_t)(size_t)sbase;
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint64_t base = ((uint64_t)hi << 32) | (uint64_t)lo;
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %2, %3\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds), "v"(voff), "s"(base)
      : "memory");
}

// Wait until at most N vector-memory operations of this wave are
// outstanding (gfx9 s_waitcnt encoding: vmcnt in bits 3:0 and 15:14; expcnt
// and lgkmcnt left at their maxima).
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// 32 bytes = 32 fp8 k-values per lane (two chunks): one 32x32x64 MFMA
// (f8f6f4 with both operands e4m3 and unit block scales).
__device__ inline void mfma_f8(f32x16& acc, const uint4& a0, const uint4& a1, const uint4& b0,
                               const uint4& b1) {
  const i32x8 av = {(int)a0.x, (int)a0.y, (int)a0.z, (int)a0.w,
                    (int)a1.x, (int)a1.y, (int)a1.z, (int)a1.w};
  const i32x8 bv = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w,
                    (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
  acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, 0, 0, 0, 127, 0, 127);
}

// float -> fp8 e4m3 byte: saturate to +-448, round to nearest even
__device__ inline uint8_t to_f8(float v) {
  v = fminf(fmaxf(v, -448.f), 448.f);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, v, 0, false) & 0xff);
}

template <typename T>
__device__ inline void store_out(const ConvArgs& a, long off, int o, float v) {
  if (a.out_f32) {
    float* p = reinterpret_cast<float*>(a.out) + off;
    if (a.accumulate) v += *p;
    *p = v;
  } else if (a.out_scale) {
    reinterpret_cast<uint8_t*>(a.out)[off] = to_f8(v * a.out_scale[o]);
  } else if constexpr (sizeof(T) == 4) {
    reinterpret_cast<float*>(a.out)[off] = v;  // FP32 nets keep fp32 activations
  } else {
    reinterpret_cast<bf16*>(a.out)[off] = (bf16)v;  // bf16, and non-fp8 outputs of fp8 layers
  }
}

template <typename T, int BM, int BN, int WM, int WN, int KB, int STAGES, int SWZ = 0>
struct Conv {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int CH = KB / 16;            // 16-byte chunks per row per step
  static constexpr int BK = KB / (int)sizeof(T);
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int TM = BM / WM, TN = BN / WN;
  static constexpr int FM = TM / 32, FN = TN / 32;
  static constexpr int A_VECS = BM * CH, B_VECS = BN * CH;
  static constexpr int A_IT = (A_VECS + NT - 1) / NT;
  static constexpr int B_IT = (B_VECS + NT - 1) / NT;
  static constexpr int LDS_BYTES = STAGES * (BM + BN) * KB;
  static_assert(FM >= 1 && FN >= 1, "wave tile >= 32x32");
  static_assert(NT % CH == 0, "chunk of a thread is fixed");
  static_assert(CH == 4 || CH == 8, "64- or 128-byte steps");
  static_assert(STAGES >= 2 && STAGES <= 4, "ring of 2 to 4 stages");
  static_assert(STAGES == 2 || (A_VECS % NT == 0 && B_VECS % NT == 0),
                "a deeper ring needs the same load count in every wave");

  // XOR key of a row: SWZ 0 makes 8 consecutive rows cover distinct 16-byte
  // bank groups of a 128-byte bank window; SWZ 1 makes 16 consecutive rows
  // distinct in a 256-byte window.
  __device__ static inline int key(int row) {
    return SWZ == 0 ? ((row / (8 / CH)) & (CH - 1)) : ((row / (16 / CH)) & (CH - 1));
  }
  // physical chunk of (row, logical chunk)
  __device__ static inline int swz(int row, int chunk) { return row * CH + (chunk ^ key(row)); }
  // the logical chunk stored at (row, physical chunk) (the XOR is an involution)
  __device__ static inline int logical_chunk(int row, int phys) { return phys ^ key(row); }
};

// Halo rows of an LDS buffer of the HALO variant: the largest
// (256/TW + 2) x (TW + 2) over the tile widths it accepts (8, 16, 32).
constexpr int kHaloRows = 340;
__host__ __device__ constexpr bool halo_width_ok(int tw) { return tw == 8 || tw == 16 || tw == 32; }

template <typename T, int BM, int BN, int WM, int WN, int KB, int STAGES, int SWZ, bool SW, bool HALO,
          bool PP = false, bool GRP = false>
__global__ __launch_bounds__(64 * WM * WN) void conv_igemm(ConvGroup ga) {
  using C = Conv<T, BM, BN, WM, WN, KB, STAGES, SWZ>;
  // GRP: several image groups; this workgroup's group (uniform) gives its
  // arguments and its range of grid x. Without GRP the arguments sit at a
  // fixed kernarg offset, so their loads need not wait for a lookup.
  int grp = 0;
  if constexpr (GRP) {
    for (int g = 1; g < ga.n; ++g)
      if ((int)blockIdx.x >= ga.first[g]) grp = g;
  }
  const ConvArgs a = ga.a[grp];  // a copy: its fields stay in registers
  static_assert(!HALO || (BM == 256 && STAGES == 2), "halo tiles: 256 pixels, two stages");
  static_assert(!PP || (HALO && BN == 256 && WM * WN == 8 && C::CH == 8),
                "two-group schedule: 256x256 halo tiles of eight waves, 128-byte steps");
  constexpr int NT = C::NT, CH = C::CH, BK = C::BK, VEC = C::VEC;
  // SW: the MFMAs take the weights as A (each lane then holds consecutive
  // channels of one pixel) and the output tile is staged through LDS for
  // 16-byte stores (bf16/fp8 outputs with 16-byte aligned channel runs);
  // otherwise the pixels are A and lanes store from registers.
  static_assert(!SW || sizeof(T) != 4, "staged epilogue: bf16 or fp8 outputs");
  constexpr int TM = C::TM, TN = C::TN, FM = C::FM, FN = C::FN;
  constexpr int A_IT = C::A_IT, B_IT = C::B_IT;
  constexpr int A_VECS = C::A_VECS, B_VECS = C::B_VECS;

  // the A/B rings, reused by the staged epilogue (BM x BN 2-byte values);
  // an A buffer holds BM rows, or a slice's halo in the HALO variant
  constexpr int AROWS = HALO ? kHaloRows : BM;
  constexpr int RING_VECS = STAGES * (AROWS + BN) * CH;
  // epilogue: the staged output tile (SW) over the rings,
  // and the 3 x BN per-channel floats past both (written before the rings
  // are released)
  constexpr int STG_VECS = SW ? BM * BN * 2 / 16 : 0;
  constexpr int PRM_OFF_VECS = STG_VECS > RING_VECS ? STG_VECS : RING_VECS;
  constexpr int SMEM_VECS = PRM_OFF_VECS + 3 * BN * 4 / 16;
  __shared__ __attribute__((aligned(16))) uint4 smem[SMEM_VECS];
  uint4 (*As)[AROWS * CH] = reinterpret_cast<uint4 (*)[AROWS * CH]>(smem);
  uint4 (*Bs)[BN * CH] = reinterpret_cast<uint4 (*)[BN * CH]>(smem + STAGES * AROWS * CH);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // uniform, so LDS destinations and per-wave offsets live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int merged = a.transposed == 2;
  // phase-grouped: the wave's column group is its phase (with two groups,
  // blockIdx.z is the phase row); uniform per wave
  const bool paired = HALO && BN == 256 && (WN == 2 || WN == 4) && a.transposed == 1;
  const int phase =
      a.transposed == 1 ? (paired ? (WN == 4 ? wn : 2 * (int)blockIdx.z + wn) : (int)blockIdx.z) : 0;
  const int py = phase >> 1, px = phase & 1;

  // XCD-aware M-tile order: consecutive workgroup ids go round-robin over
  // the 8 XCDs; give each XCD a contiguous range of tiles.
  const int gx = GRP ? ga.first[grp + 1] - ga.first[grp] : (int)gridDim.x;
  const int bx = GRP ? (int)blockIdx.x - ga.first[grp] : (int)blockIdx.x;
  const int xcd = bx & 7, q = gx >> 3, r = gx & 7;
  const int mt = xcd * q + min(xcd, r) + (bx >> 3);

  // 2-D M tile: image, tile row, tile column
  const int TW = a.tile_w, TH = BM / a.tile_w;
  const int tiles_x = (a.Wo + TW - 1) / TW, tiles_y = (a.Ho + TH - 1) / TH;
  const int img_t = mt / (tiles_x * tiles_y);
  const int rem_t = mt - img_t * tiles_x * tiles_y;
  const int ty0 = (rem_t / tiles_x) * TH, tx0 = (rem_t % tiles_x) * TW;
  const int n0 = blockIdx.y * BN;
  // output channel of this wave's first column (paired: within its phase)
  const int col0 = paired ? 0 : n0 + wn * TN;
  // The tile's per-channel parameters (bias, weight scale, fp8 output
  // scale) of channels pbase .. pbase + BN - 1, one channel per thread:
  // loaded now, so the loads complete under the main loop, and put in LDS
  // after it.
  static_assert(NT >= BN, "one parameter channel per thread");
  const int pbase = (merged || paired) ? 0 : n0;
  float pv[3] = {0.f, 1.f, 1.f};
  if (tid < BN) {
    const int n = pbase + tid;
    if (n < a.cout) {
      pv[0] = a.bias[n];
      if (a.w_scale) pv[1] = a.w_scale[n];
      if (a.out_scale) pv[2] = a.out_scale[n];
    }
  }
  const int chunk = tid % CH;  // this thread's chunk within a row

  const T* in = reinterpret_cast<const T*>(a.in);
  const T* wgt = reinterpret_cast<const T*>(a.wgt);
  (void)VEC;

  // a step stays inside one tap when the channel count is a multiple of BK
  const bool tap_uniform = (a.cin_pad % BK) == 0;
  // input offset of tap t: 3x3 neighbourhood, or the 2x2 taps of one
  // transposed-conv output phase
  auto tap_dy = [&](int t) { return a.transposed == 1 ? py - (t >> 1) : ((t * 11) >> 5) - 1; };
  auto tap_dx = [&](int t) {
    return a.transposed == 1 ? px - (t & 1) : t - 3 * (((t * 11) >> 5)) - 1;
  };

  // Per A-load data, fixed across the K loop. Load i of this thread fills
  // LDS slot tid + i*NT = (row, physical chunk tid % CH): the pixel's offset
  // in its image, a bit mask of the taps whose sample lies inside the image
  // (none for rows past the grid), and for tap-major K order the running
  // (tap, channel) of this load's k.
  const T* a_ptr[A_IT];
  int a_pix[A_IT], a_tap[A_IT], a_c[A_IT];
  uint32_t a_mask[A_IT];
#pragma unroll
  for (int i = 0; i < (HALO ? 0 : A_IT); ++i) {
    const int v = tid + i * NT;
    const int row = v / CH;
    const int oy = ty0 + row / TW, ox = tx0 + row % TW;
    const bool ok = (v < A_VECS) && (oy < a.Ho) && (ox < a.Wo);
    const int iy0 = oy * a.stride, ix0 = ox * a.stride;
    const int kk = C::logical_chunk(row, chunk) * VEC;
    a_ptr[i] = in + (long)img_t * a.in_img_stride + (tap_uniform ? kk : 0);
    a_pix[i] = (iy0 * a.Wi + ix0) * a.in_ld;
    uint32_t m = 0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int iy = iy0 + tap_dy(t), ix = ix0 + tap_dx(t);
      if (ok && t < a.taps && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi) m |= 1u << t;
    }
    a_mask[i] = m;
    a_tap[i] = kk / a.cin_pad;
    a_c[i] = kk - a_tap[i] * a.cin_pad;
  }
  // HALO: load i of a slice fills halo slot tid + i*NT = (halo row, physical
  // chunk); h_off is its input offset in the image (-1: outside the image
  // or past the halo); hb[i] the halo row of fragment i's pixel at tap
  // offset (0, 0).
  constexpr int HA_IT = HALO ? (kHaloRows * CH + NT - 1) / NT : 1;
  const int hwid = a.tile_w + 2;
  // hrow / hwid as (hrow * hw_mul) >> 16: exact for the halo rows (< 400)
  const int hw_mul = (65536 + hwid - 1) / hwid;
  const int h_vecs = (BM / a.tile_w + 2) * hwid * CH;
  int h_off[HA_IT];
  int hb[FM];
  if constexpr (HALO) {
#pragma unroll
    for (int i = 0; i < HA_IT; ++i) {
      const int v = tid + i * NT;
      const int hrow = v / CH;
      const int iy = ty0 - 1 + hrow / hwid, ix = tx0 - 1 + hrow % hwid;
      const bool ok = v < h_vecs && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
      h_off[i] = ok ? (iy * a.Wi + ix) * a.in_ld + C::logical_chunk(hrow, chunk) * VEC : -1;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int p = wm * TM + i * 32 + (lane & 31);
      hb[i] = (p / TW + 1) * hwid + p % TW + 1;
    }
  }
  const T* b_ptr[B_IT];
#pragma unroll
  for (int i = 0; i < B_IT; ++i) {
    const int v = tid + i * NT;
    const int row = (B_VECS % NT == 0 || v < B_VECS) ? v / CH : 0;
    // packed weights are [phase][cout_pad][K_pad]; phase-grouped tiles
    // stack row r % TN of the r / TN-th phase of the group at tile row r
    const long prow = paired ? (long)((WN == 4 ? 0 : 2 * (int)blockIdx.z) + row / TN) * a.cout_pad + row % TN
                             : (long)(a.transposed == 1 ? (int)blockIdx.z : 0) * a.cout_pad + n0 + row;
    b_ptr[i] = wgt + prow * a.K_pad + C::logical_chunk(row, chunk) * VEC;
  }
  const T* zero = reinterpret_cast<const T*>(a.zero);
  const int nk = a.K_pad / BK;
  const int lrow = lane & 31;
  const int lhalf = lane >> 5;
  const int step_taps = BK / a.cin_pad, step_c = BK - step_taps * a.cin_pad;

  // Issue the loads of K step kc into ring buffer buf. Steps are issued in
  // increasing order, one at a time (the tap-major counters advance here).
  const T* in_img = in + (long)img_t * a.in_img_stride;
  // HALO: the weight tile of step kc, and the halo loads of slice `slice`
  // whose index is congruent to `part` modulo the tap count (part < 0: all)
  auto issue_b = [&](int kc, int buf) {
#pragma unroll
    for (int i = 0; i < B_IT; ++i) {
      const T* src = b_ptr[i] + (long)kc * BK;
      if (B_VECS % NT == 0 || tid + i * NT < B_VECS) load_to_lds(src, &Bs[buf][i * NT + wave * 64]);
    }
  };
  auto issue_halo = [&](int slice, int buf, int part) {
#pragma unroll
    for (int i = 0; i < HA_IT; ++i) {
      if (part >= 0 && i % a.taps != part) continue;
      if (i * NT >= h_vecs) continue;
      const T* src = h_off[i] >= 0 ? in_img + (h_off[i] + slice * BK) : zero;
      if (tid + i * NT < h_vecs) load_to_lds(src, &As[buf][i * NT + wave * 64]);
    }
  };

  auto issue = [&](int kc, int buf) {
    if (tap_uniform) {
      // channel-slice major: all taps of a BK-channel slice back to back, so
      // the input lines of a slice are reused while still in L2 (the packed
      // weights use the same order); tap and slice are uniform
      const int slice = kc / a.taps;
      const int tap = kc - slice * a.taps;
      const int c_u = slice * BK;
      const bool kin = c_u < a.cin_pad;  // steps past the real K read nothing
      const int toff = (tap_dy(tap) * a.Wi + tap_dx(tap)) * a.in_ld + c_u;
#pragma unroll
      for (int i = 0; i < A_IT; ++i) {
        const bool ok = kin && ((a_mask[i] >> tap) & 1u);
        const T* src = ok ? a_ptr[i] + (a_pix[i] + toff) : zero;
        if (A_VECS % NT == 0 || tid + i * NT < A_VECS) load_to_lds(src, &As[buf][i * NT + wave * 64]);
      }
    } else {
      // tap major: a step spans several taps; each load follows its own k
#pragma unroll
      for (int i = 0; i < A_IT; ++i) {
        const int tap = a_tap[i];  // >= taps once k passes the real K: mask bit 0
        const bool ok = (a_mask[i] >> tap) & 1u;
        const int toff = (tap_dy(tap) * a.Wi + tap_dx(tap)) * a.in_ld + a_c[i];
        const T* src = ok ? a_ptr[i] + (a_pix[i] + toff) : zero;
        if (A_VECS % NT == 0 || tid + i * NT < A_VECS) load_to_lds(src, &As[buf][i * NT + wave * 64]);
        a_c[i] += step_c;
        a_tap[i] += step_taps;
        if (a_c[i] >= a.cin_pad) {
          a_c[i] -= a.cin_pad;
          a_tap[i] += 1;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < B_IT; ++i) {
      const T* src = b_ptr[i] + (long)kc * BK;
      if (B_VECS % NT == 0 || tid + i * NT < B_VECS) load_to_lds(src, &Bs[buf][i * NT + wave * 64]);
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // A fragment row of fragment i: the tile row, or (HALO) the halo row of
  // the pixel shifted by this step's tap offset hoff
  auto arow = [&](int i, int hoff) { return HALO ? hb[i] + hoff : wm * TM + i * 32 + lrow; };
  auto compute = [&](int buf, int abuf, int hoff) {
    if constexpr (sizeof(T) == 1) {
      // fp8: a lane half's CH/2 chunks feed CH/4 MFMAs of two chunks each
#pragma unroll
      for (int s = 0; s < CH / 4; ++s) {
        const int ch = lhalf * (CH / 2) + 2 * s;
        uint4 fa[FM][2], fb[FN][2];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          fa[i][0] = As[abuf][C::swz(arow(i, hoff), ch)];
          fa[i][1] = As[abuf][C::swz(arow(i, hoff), ch + 1)];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          fb[j][0] = Bs[buf][C::swz(wn * TN + j * 32 + lrow, ch)];
          fb[j][1] = Bs[buf][C::swz(wn * TN + j * 32 + lrow, ch + 1)];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (SW)
              mfma_f8(acc[i][j], fb[j][0], fb[j][1], fa[i][0], fa[i][1]);
            else
              mfma_f8(acc[i][j], fa[i][0], fa[i][1], fb[j][0], fb[j][1]);
          }
      }
    } else {
#pragma unroll
      for (int s = 0; s < CH / 2; ++s) {
        const int ch = lhalf * (CH / 2) + s;
        uint4 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = As[abuf][C::swz(arow(i, hoff), ch)];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = Bs[buf][C::swz(wn * TN + j * 32 + lrow, ch)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (SW)
              mfma_chunk<T>(acc[i][j], fb[j], fa[i]);
            else
              mfma_chunk<T>(acc[i][j], fa[i], fb[j]);
          }
      }
    }
  };

  // Ring of STAGES buffers: the loads of steps k+1 .. k+STAGES-1 are in
  // flight while step k computes. The LDS loads are issued outside the
  // compiler's view, so the waits for them are explicit: before the barrier
  // of step k, at most the loads of the younger steps may be outstanding
  // (vmcnt drains in issue order).
  if constexpr (PP) {
    // Two-group schedule. Waves 0-3 (group 0) and 4-7 (group 1) hold one
    // wave of each group per SIMD; every step k is a memory phase M_k (all
    // of the step's fragments read from LDS into registers, plus this
    // group's share of future global->LDS loads) and a compute phase C_k
    // (the step's MFMAs only), each ended by a workgroup barrier. Group 1
    // runs one barrier behind group 0, so on every SIMD one wave's MFMAs
    // overlap the other wave's LDS reads and load issue.
    //   barrier numbers: group 0 runs M_k between barriers 2k-1 and 2k and
    //   C_k up to 2k+1; group 1 runs M_k up to 2k+1 and C_k up to 2k+2.
    //   Weights: group 0 issues step k+1's tile in M_k into buffer (k+1)&1,
    //   which group 1 last read in M_{k-1} (done by barrier 2k-1), and waits
    //   for it before barrier 2k+1, ahead of both groups' M_{k+1}.
    //   Halo: group 1 issues the next slice's halo in the slice's first
    //   taps-1 steps (piece i in tap step i mod (taps-1)) into the buffer
    //   the previous slice used (last read in group 1's M of that slice's
    //   final step), and waits for each piece before the barrier closing
    //   its following C phase, ahead of group 0's first M of the next slice.
    //   (Issuing the loads between the MFMA rounds of a C phase instead
    //   measured 6 % slower.)
    const int n_slices = a.cin_pad / BK;
    const int grp = wave >> 2;
    const int gw = wave & 3;             // wave within its group
    const int gtid = tid & 255;          // thread within its group
    const int gchunk = gtid & (CH - 1);  // this thread's physical chunk
    constexpr int RCH = sizeof(T) == 1 ? 2 : 1;  // chunks per MFMA round
    constexpr int NR = CH / 2 / RCH;              // rounds per step
    constexpr int BPT = BN * CH / 256;            // weight loads of a step per group-0 thread
    // weight rows r0 + 32 i of the B tile (r0 = gtid / CH): their XOR key
    // does not depend on i, so one lane offset serves every load and the
    // row and step offsets are uniform
    const int r0 = gtid / CH;
    const uint32_t b_voff = (uint32_t)((r0 * a.K_pad + C::logical_chunk(r0, gchunk) * VEC) * (int)sizeof(T));
    auto brow0 = [&](int i) -> long {  // packed-weight row of B-tile row 32 i
      const int row = 32 * i;
      return paired ? (long)((WN == 4 ? 0 : 2 * (int)blockIdx.z) + row / TN) * a.cout_pad + row % TN
                    : (long)(a.transposed == 1 ? (int)blockIdx.z : 0) * a.cout_pad + n0 + row;
    };
    // weight loads i0 .. i1-1 of step kc's tile into buffer buf
    auto issue_b_pp = [&](int kc, int buf, int i0, int i1) {
#pragma unroll
      for (int i = i0; i < i1; ++i)
        load_to_lds_s(wgt + brow0(i) * a.K_pad + (long)kc * BK, b_voff, &Bs[buf][i * 256 + gw * 64]);
    };
    const int n_pieces = (h_vecs + 255) / 256;
    auto issue_halo_piece = [&](int slice, int buf, int i) {
      const int v = gtid + i * 256;
      const int hrow = v / CH;
      const int hy = (hrow * hw_mul) >> 16, hx = hrow - hy * hwid;
      const int iy = ty0 - 1 + hy, ix = tx0 - 1 + hx;
      const bool ok = v < h_vecs && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
      const T* src = ok ? in_img + ((iy * a.Wi + ix) * a.in_ld + C::logical_chunk(hrow, gchunk) * VEC +
                                    slice * BK)
                        : zero;
      if (v < h_vecs) load_to_lds(src, &As[buf][i * 256 + gw * 64]);
    };
    if (grp == 0) {
      issue_b_pp(0, 0, 0, BPT);
      if (nk > 1) issue_b_pp(1, 1, 0, BPT);
    } else if (n_slices > 0) {
      for (int i = 0; i < n_pieces; ++i) issue_halo_piece(0, 0, i);
    }
    wait_vm<0>();
    __syncthreads();
    if (grp == 1) __syncthreads();
    const int hsteps = a.taps - 1;  // tap steps of a slice that issue halo pieces
    for (int kc = 0; kc < nk; ++kc) {
      const int slice = kc / a.taps, tap = kc - slice * a.taps;
      const int buf = kc & 1, abuf = slice & 1;
      const int hoff = tap_dy(tap) * hwid + tap_dx(tap);
      // M_k: every fragment of the step, then this group's loads
      uint4 fa[NR][FM][RCH], fb[NR][FN][RCH];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < RCH; ++c) {
          const int ch = lhalf * (CH / 2) + r * RCH + c;
#pragma unroll
          for (int i = 0; i < FM; ++i) fa[r][i][c] = As[abuf][C::swz(arow(i, hoff), ch)];
#pragma unroll
          for (int j = 0; j < FN; ++j) fb[r][j][c] = Bs[buf][C::swz(wn * TN + j * 32 + lrow, ch)];
        }
      if (grp == 0) {
        if (kc >= 1 && kc + 1 < nk) issue_b_pp(kc + 1, (kc + 1) & 1, 0, BPT);
      } else if (slice + 1 < n_slices && tap < hsteps) {
        for (int i = tap; i < n_pieces; i += hsteps) issue_halo_piece(slice + 1, (slice + 1) & 1, i);
      }
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      // C_k: the step's MFMAs
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (sizeof(T) == 1) {
              if constexpr (SW)
                mfma_f8(acc[i][j], fb[r][j][0], fb[r][j][1], fa[r][i][0], fa[r][i][1]);
              else
                mfma_f8(acc[i][j], fa[r][i][0], fa[r][i][1], fb[r][j][0], fb[r][j][1]);
            } else {
              if constexpr (SW)
                mfma_chunk<T>(acc[i][j], fb[r][j][0], fa[r][i][0]);
              else
                mfma_chunk<T>(acc[i][j], fa[r][i][0], fb[r][j][0]);
            }
          }
      __builtin_amdgcn_sched_barrier(0);
      wait_vm<0>();
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
    }
    if (grp == 0) __syncthreads();
  } else if constexpr (HALO) {
    // two weight stages and two halo buffers; every load of step kc is
    // waited for (vmcnt 0) before the barrier of step kc + 1. Inside a step
    // the fragments of round r + 1 are read while round r's MFMAs run, and
    // the first round's reads go out before the next step's loads are
    // issued, so the MFMAs start as early as the data allows.
    const int n_slices = a.cin_pad / BK;
    constexpr int RCH = sizeof(T) == 1 ? 2 : 1;  // chunks per MFMA round
    constexpr int NR = CH / 2 / RCH;              // rounds per step
    issue_b(0, 0);
    if (n_slices > 0) issue_halo(0, 0, -1);
    for (int kc = 0; kc < nk; ++kc) {
      wait_vm<0>();
      __syncthreads();
      const int slice = kc / a.taps, tap = kc - slice * a.taps;
      const int buf = kc & 1, abuf = slice & 1;
      const int hoff = tap_dy(tap) * hwid + tap_dx(tap);
      uint4 fa[2][FM][RCH], fb[2][FN][RCH];
      auto read_round = [&](int r, uint4 (&xa)[FM][RCH], uint4 (&xb)[FN][RCH]) {
#pragma unroll
        for (int c = 0; c < RCH; ++c) {
          const int ch = lhalf * (CH / 2) + r * RCH + c;
#pragma unroll
          for (int i = 0; i < FM; ++i) xa[i][c] = As[abuf][C::swz(arow(i, hoff), ch)];
#pragma unroll
          for (int j = 0; j < FN; ++j) xb[j][c] = Bs[buf][C::swz(wn * TN + j * 32 + lrow, ch)];
        }
      };
      read_round(0, fa[0], fb[0]);
      if (kc + 1 < nk) issue_b(kc + 1, (kc + 1) & 1);
      if (slice + 1 < n_slices) {
        // this tap's share of the next slice's halo: slots tid + i*NT,
        // i = tap and tap + taps (per-phase convs have 4 taps, 6 pieces)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int i = tap + k * a.taps;
          if (i * NT < h_vecs) {
            const int v = tid + i * NT;
            const int hrow = v / CH;
            const int hy = (hrow * hw_mul) >> 16, hx = hrow - hy * hwid;
            const int iy = ty0 - 1 + hy, ix = tx0 - 1 + hx;
            const bool ok = v < h_vecs && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
            const T* src = ok ? in_img + ((iy * a.Wi + ix) * a.in_ld + C::logical_chunk(hrow, chunk) * VEC +
                                          (slice + 1) * BK)
                              : zero;
            if (v < h_vecs) load_to_lds(src, &As[(slice + 1) & 1][i * NT + wave * 64]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int cur = r & 1;
        if (r + 1 < NR) read_round(r + 1, fa[cur ^ 1], fb[cur ^ 1]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (sizeof(T) == 1) {
              if constexpr (SW)
                mfma_f8(acc[i][j], fb[cur][j][0], fb[cur][j][1], fa[cur][i][0], fa[cur][i][1]);
              else
                mfma_f8(acc[i][j], fa[cur][i][0], fa[cur][i][1], fb[cur][j][0], fb[cur][j][1]);
            } else {
              if constexpr (SW)
                mfma_chunk<T>(acc[i][j], fb[cur][j][0], fa[cur][i][0]);
              else
                mfma_chunk<T>(acc[i][j], fa[cur][i][0], fb[cur][j][0]);
            }
          }
      }
    }
  } else {
    constexpr int LPS = A_IT + B_IT;  // loads per step per thread
#pragma unroll
    for (int st = 0; st < STAGES - 1; ++st)
      if (st < nk) issue(st, st);
    for (int kc = 0; kc < nk; ++kc) {
      if (kc + STAGES - 2 < nk)
        wait_vm<(STAGES - 2) * LPS>();
      else
        wait_vm<0>();
      __syncthreads();
      if (kc + STAGES - 1 < nk) issue(kc + STAGES - 1, (kc + STAGES - 1) % STAGES);
      compute(kc % STAGES, kc % STAGES, 0);
    }
  }

  // The per-channel parameters go to their own LDS area (outside the rings
  // and the staging area); the barrier that releases the rings makes them
  // visible to every wave.
  float* prm = reinterpret_cast<float*>(smem + PRM_OFF_VECS);
  if (tid < BN) {
    prm[tid] = pv[0];
    prm[BN + tid] = pv[1];
    prm[2 * BN + tid] = pv[2];
  }
  __syncthreads();

  if constexpr (!SW) {
    // Epilogue (pixels as A): lane l holds channel l%32 of fragment j for 16
    // pixels; bias, ReLU, optional accumulate, store (NHWC, channel slice).
    const int cout_m = merged ? a.cout : 1;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      long off_row[16];
      bool row_ok[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wm * TM + i * 32 + (e >> 2) * 8 + lhalf * 4 + (e & 3);
        int oy = ty0 + row / TW;
        int ox = tx0 + row % TW;
        row_ok[e] = oy < a.Ho && ox < a.Wo;
        if (a.transposed) {  // output of the GEMM grid point (oy, ox), phase (0, 0)
          oy *= 2;
          ox *= 2;
        }
        off_row[e] = (long)img_t * a.out_img_stride + ((long)(oy + py) * a.Wout + ox + px) * a.out_ld;
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = col0 + j * 32 + lrow;
        long col;
        int o;
        if (!merged) {
          if (n >= a.cout) continue;
          o = n;
          col = n;
        } else {
          if (n >= 4 * cout_m) continue;
          const int ph = n / cout_m;
          o = n - ph * cout_m;
          col = ((long)(ph >> 1) * a.Wout + (ph & 1)) * a.out_ld + o;
        }
        const float bn = prm[o - pbase];
        const float ws = prm[BN + o - pbase];
        float amax = 0.f;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          if (!row_ok[e]) continue;
          float v = acc[i][j][e] * ws + bn;
          if (a.relu) v = fmaxf(v, 0.f);
          amax = fmaxf(amax, fabsf(v));
          store_out<T>(a, off_row[e] + col, o, v);
        }
        if (a.amax) atomicMax(reinterpret_cast<unsigned*>(a.amax) + o, __float_as_uint(amax));
      }
    }
  } else {
    // Epilogue (weights as A): lane l holds, for fragment (i, j), pixel
    // i*32 + l%32 of the wave tile and channels j*32 + 8g + 4*(l/32) + q
    // (g, q = 0..3). Bias, scale and ReLU are applied in registers; the
    // wave's TM x TN output tile is written to its own LDS region (rows
    // XOR-swizzled in 16-byte chunks) and read back row by row, so each
    // global store moves 16 contiguous bytes per lane and whole pixel rows
    // per group of lanes.
    const int E = a.out_scale ? 1 : 2;  // output element bytes (fp8 or bf16)
    {
      char* region = reinterpret_cast<char*>(smem) + (size_t)wave * TM * TN * 2;
      // Channel-group major, so only one group's bias and scale are live.
      // A wave64 VALU instruction takes four cycles, so this loop (128
      // values per lane) is specialised on the uniform flags: ReLU, output
      // type and (calibration only) the running |max|, with no per-value
      // branch; bf16 pairs convert with one instruction.
      auto convert = [&](auto relu_c, auto e_c, auto amax_c) {
        constexpr bool RELU = decltype(relu_c)::value, AMAX = decltype(amax_c)::value;
        constexpr int EE = decltype(e_c)::value;
        constexpr int PITCH = TN * EE, CPR = PITCH / 16;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int c0 = j * 32 + 8 * g + 4 * lhalf;  // channel within the wave tile
            const int n = col0 + c0;
            const float* pc = prm + (n - pbase);  // in [0, BN), 16-byte aligned
            const float4 bias4 = *reinterpret_cast<const float4*>(pc);
            const float4 ws4 = *reinterpret_cast<const float4*>(pc + BN);
            const float bq[4] = {bias4.x, bias4.y, bias4.z, bias4.w};
            const float sq[4] = {ws4.x, ws4.y, ws4.z, ws4.w};
            float os[4] = {1.f, 1.f, 1.f, 1.f};
            if constexpr (EE == 1) {
              const float4 o4 = *reinterpret_cast<const float4*>(pc + 2 * BN);
              os[0] = o4.x, os[1] = o4.y, os[2] = o4.z, os[3] = o4.w;
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
              const int p = i * 32 + lrow;
              float v[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                float x = acc[i][j][4 * g + q] * sq[q] + bq[q];
                if constexpr (RELU) x = fmaxf(x, 0.f);
                v[q] = x;
              }
              if constexpr (AMAX) {
                if (n < a.cout)  // cout is a multiple of 8: all four or none
#pragma unroll
                  for (int q = 0; q < 4; ++q)
                    atomicMax(reinterpret_cast<unsigned*>(a.amax) + n + q, __float_as_uint(fabsf(v[q])));
              }
              const int byte = c0 * EE;
              const int chunk = (byte >> 4) ^ (p & (CPR - 1));
              char* dst = region + p * PITCH + chunk * 16 + (byte & 15);
              if constexpr (EE == 2) {
                uint2 w;
                w.x = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[0], v[1]}, bf16x2));
                w.y = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[2], v[3]}, bf16x2));
                *reinterpret_cast<uint2*>(dst) = w;
              } else {
                uint32_t w = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) w |= (uint32_t)to_f8(v[q] * os[q]) << (8 * q);
                *reinterpret_cast<uint32_t*>(dst) = w;
              }
            }
          }
        }
      };
      using T0 = std::false_type;
      using T1 = std::true_type;
      using E1 = std::integral_constant<int, 1>;
      using E2 = std::integral_constant<int, 2>;
      if (a.amax) {
        if (E == 2) {
          if (a.relu) convert(T1{}, E2{}, T1{});
          else convert(T0{}, E2{}, T1{});
        } else {
          if (a.relu) convert(T1{}, E1{}, T1{});
          else convert(T0{}, E1{}, T1{});
        }
      } else if (E == 2) {
        if (a.relu) convert(T1{}, E2{}, T0{});
        else convert(T0{}, E2{}, T0{});
      } else {
        if (a.relu) convert(T1{}, E1{}, T0{});
        else convert(T0{}, E1{}, T0{});
      }
      __syncthreads();  // the region is read back by other lanes of the wave
      // Read-back: lane l takes chunk l % CPR of wave-tile rows l / CPR +
      // R * it (R = 64 / CPR rows per step). Every chunk is read from LDS
      // first, then stored; the output position advances by R rows per step
      // without a division.
      auto flush = [&](auto cpr_c) {
        constexpr int CPR = decltype(cpr_c)::value;
        constexpr int R = 64 / CPR, IT = TM / R;
        const int ch = lane % CPR, p_l = lane / CPR;
        uint4 w[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          const int p = p_l + R * it;
          w[it] = *reinterpret_cast<const uint4*>(region + p * (CPR * 16) + ((ch ^ (p & (CPR - 1))) * 16));
        }
        // every read is issued before the first store waits for them
#pragma unroll
        for (int it = 0; it < IT; ++it) asm volatile("" ::"v"(w[it].x), "v"(w[it].y), "v"(w[it].z), "v"(w[it].w));
        const int n = col0 + ch * (16 / E);
        if (n >= a.cout) return;
        const int row0 = wm * TM + p_l;
        int ry = row0 / TW, rx = row0 - ry * TW;  // row within the M tile's TH x TW block
        const int dy = R / TW, dx = R - dy * TW;  // R rows further (uniform)
        char* out = reinterpret_cast<char*>(a.out);
        const long img_off = (long)img_t * a.out_img_stride + n;
        const int sh = a.transposed ? 1 : 0;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          const int oy = ty0 + ry, ox = tx0 + rx;
          if (oy < a.Ho && ox < a.Wo) {
            const int q = ((oy << sh) + py) * a.Wout + (ox << sh) + px;  // output pixel
            *reinterpret_cast<uint4*>(out + (img_off + (long)q * a.out_ld) * E) = w[it];
          }
          rx += dx;
          ry += dy;
          if (rx >= TW) {
            rx -= TW;
            ++ry;
          }
        }
      };
      if (E == 2)
        flush(std::integral_constant<int, TN * 2 / 16>{});
      else
        flush(std::integral_constant<int, TN / 16>{});
    }
  }
}

// Whether the HALO variant covers a launch: a stride-1 3x3 neighbourhood
// (plain, per-phase transposed with 4 taps, or phase-merged), channel
// slices that are whole K steps in slice-major K order, and a tile width
// whose halo fits the buffer.
inline bool halo_tile_ok(const ConvArgs& a, int bk) {
  const bool nb = (a.transposed == 0 && a.stride == 1 && a.taps == 9) ||
                  (a.transposed == 1 && a.taps == 4) || (a.transposed == 2 && a.taps == 9);
  return nb && a.cin_pad % bk == 0 && a.K_pad == a.taps * a.cin_pad && a.Hi == a.Ho && a.Wi == a.Wo &&
         halo_width_ok(a.tile_w);
}

template <typename T, int BM, int BN, int WM, int WN, int KB, int STAGES, int SWZ = 0, bool HALO = false,
          bool PP = false>
hipError_t launch_variant(const ConvArgs* args, int n_groups, hipStream_t s) {
  using C = Conv<T, BM, BN, WM, WN, KB, STAGES, SWZ>;
  if (n_groups < 1 || n_groups > ConvGroup::kMax) return hipErrorInvalidValue;
  ConvGroup ga{};
  ga.n = n_groups;
  long total = 0;
  const ConvArgs& a0 = args[0];
  // phase-grouped 256-column HALO tiles: WN phases per workgroup
  const bool paired = HALO && BN == 256 && (WN == 2 || WN == 4) && a0.transposed == 1;
  for (int g = 0; g < n_groups; ++g) {
    const ConvArgs& a = args[g];
    if (HALO && !halo_tile_ok(a, C::BK)) return hipErrorInvalidValue;
    if (paired && (a.n_rows > BN / WN || a.cout_pad < BN / WN)) return hipErrorInvalidValue;
    const int n_tiles = paired ? 1 : (a.n_rows + BN - 1) / BN;
    // every B row a tile reads (n_tiles * BN of them) must exist in the packed weights
    if (a.K_pad % C::BK != 0 || a.cin_pad % C::VEC != 0 || a.n_rows <= 0 ||
        n_tiles * BN > a.cout_pad || a.in_ld % C::VEC != 0 || a.tile_w <= 0 || BM % a.tile_w != 0)
      return hipErrorInvalidValue;
    // the groups share the layer: channels, mode and output layout
    if (a.transposed != a0.transposed || a.n_rows != a0.n_rows || a.cout != a0.cout || a.taps != a0.taps ||
        a.out_f32 != a0.out_f32 || a.out_ld != a0.out_ld || (a.out_scale == nullptr) != (a0.out_scale == nullptr))
      return hipErrorInvalidValue;
    // per-image input offsets are 32-bit in the kernel
    if ((long)a.Hi * a.Wi * a.in_ld >= (1L << 31)) return hipErrorInvalidValue;
    const long tiles = (long)a.n_img * ((a.Ho + BM / a.tile_w - 1) / (BM / a.tile_w)) *
                       ((a.Wo + a.tile_w - 1) / a.tile_w);
    ga.a[g] = a;
    ga.first[g] = (int)total;
    total += tiles;
    if (total > 0x7fffffffL) return hipErrorInvalidValue;
  }
  ga.first[n_groups] = (int)total;
  if (total == 0) return hipSuccess;
  const int phases = a0.transposed == 1 ? (paired ? 4 / WN : 4) : 1;
  const int n_tiles = paired ? 1 : (a0.n_rows + BN - 1) / BN;
  dim3 grid((unsigned)total, (unsigned)n_tiles, phases);
  // the staged epilogue needs bf16/fp8 outputs in 16-byte channel runs
  const int run = a0.out_scale ? 16 : 8;
  const bool staged = sizeof(T) != 4 && BN >= 32 && a0.transposed != 2 && !a0.out_f32 &&
                      a0.cout % run == 0 && a0.out_ld % run == 0;
  if (n_groups > 1) {
    // grouped launches: the generic tiles and the two-group halo tile
    if constexpr (!HALO || PP) {
      if constexpr (sizeof(T) != 4 && BN >= 32) {
        if (staged) {
          hipLaunchKernelGGL((conv_igemm<T, BM, BN, WM, WN, KB, STAGES, SWZ, true, HALO, PP, true>), grid,
                             dim3(C::NT), 0, s, ga);
          return hipGetLastError();
        }
      }
      hipLaunchKernelGGL((conv_igemm<T, BM, BN, WM, WN, KB, STAGES, SWZ, false, HALO, PP, true>), grid,
                         dim3(C::NT), 0, s, ga);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if constexpr (sizeof(T) != 4 && BN >= 32) {
    if (staged) {
      hipLaunchKernelGGL((conv_igemm<T, BM, BN, WM, WN, KB, STAGES, SWZ, true, HALO, PP>), grid, dim3(C::NT),
                         0, s, ga);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((conv_igemm<T, BM, BN, WM, WN, KB, STAGES, SWZ, false, HALO, PP>), grid, dim3(C::NT), 0,
                     s, ga);
  return hipGetLastError();
}

}  // namespace convk
}  // namespace ffv
