// Persistent halo-reuse convolution with the weights resident in LDS, for
// layers with few output channels over a stride-1 3x3 neighbourhood whose
// whole weight matrix fits next to two input halos (supplementary layer
// table: the flow/mask heads of the VIBlocks, phase-merged 4x4 transposed
// convs, and the stride-1 3x3 convs of the narrow U-Net levels), and for
// one output phase of a 4x4 stride-2 transposed conv (four 2x2 taps over
// the same neighbourhood; a workgroup keeps one phase's weights).
//
// These layers have one or two channel slices per output block, so a
// kernel that loads each block's input and weights and then computes has
// nothing to hide the load latency behind: one slice's MFMAs are a few
// hundred cycles, one load round trip from HBM several thousand. Here a
// workgroup stays resident on its compute unit, loads the weights once, and
// walks a range of 16x16 output blocks with one pipeline of channel-slice
// steps that runs across block boundaries: while it computes the last slice
// of a block, the first slice's halo of its next block is already loading,
// and the block's epilogue (registers straight to global memory) overlaps
// that load as well. Every tap reads its shifted window of the halo from
// LDS (as in the non-resident halo kernel), and its weights from the
// resident copy.
#pragma once

#include <type_traits>

#include "conv_halo.h"

namespace ffv {
namespace convk {

struct Resident {
  static constexpr int NT = 512;                     // 8 waves
  static constexpr int TW = 16, TH = 16;             // output block
  static constexpr int HW = TW + 2;                  // halo row width
  static constexpr int NH = HW * (TH + 2);           // halo pixels
  static constexpr int KB = 128;                     // bytes of a pixel's channel slice
  static constexpr int CH = KB / 16;
  static constexpr int A_VECS = NH * CH;
  static constexpr int A_IT = (A_VECS + NT - 1) / NT;
  // resident weights: BN rows of K_pad values, 16-byte chunks, row pitch
  // one chunk longer than the row (odd pitch: the 32 rows a fragment read
  // touches fall in distinct bank groups, 16 at a time)
  static constexpr int W_VECS = 4800;
};

// Whether the resident kernel with an N tile of bn channels covers a launch
// (the weights of every output channel must fit the resident buffer).
inline bool resident_ok(const ConvArgs& a, int bn, int elem_bytes) {
  const int bk = Resident::KB / elem_bytes;
  const bool nb = (a.transposed == 0 && a.stride == 1 && a.taps == 9) || (a.transposed == 2 && a.taps == 9) ||
                  (a.transposed == 1 && a.taps == 4);
  const long row_bytes = (long)a.K_pad * elem_bytes;
  if (!nb || a.cin_pad % bk != 0 || a.K_pad != a.taps * a.cin_pad || row_bytes % 16 != 0) return false;
  const long rc = row_bytes / 16;
  return a.Hi == a.Ho && a.Wi == a.Wo && a.n_rows <= bn && bn <= a.cout_pad &&
         bn * (rc + 1) <= Resident::W_VECS && a.tile_w == Resident::TW;
}

// Two waves per SIMD is all the LDS footprint allows; saying so lets the
// compiler keep a second tap's fragments in registers. EPI 1 and 2: the
// weights are the MFMA's A operand, so a lane ends with runs of 4
// consecutive GEMM columns of one pixel, and the epilogue stages each
// wave's 32 x BN output tile through LDS: EPI 1 for bf16/fp8 outputs in
// 16-byte channel runs (16-byte stores), EPI 2 for float outputs of a
// 32-column tile (one lane per output pixel, float4 accesses, in-place
// accumulation). EPI 0: lanes store single values from registers.
// TAPS 4: one output phase of a transposed conv per workgroup.
template <typename T, int BN, int EPI, int TAPS>
__global__ __launch_bounds__(Resident::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void conv_resident(ConvArgs a, int n_tiles) {
  constexpr bool SW = EPI != 0;
  static_assert(EPI != 2 || BN == 32, "float staging holds 32-column tiles");
  using R = Resident;
  constexpr int NT = R::NT, CH = R::CH, TW = R::TW, TH = R::TH, HW = R::HW;
  constexpr int A_IT = R::A_IT, A_VECS = R::A_VECS, FN = BN / 32;
  constexpr int BK = R::KB / (int)sizeof(T), VEC = 16 / (int)sizeof(T);

  __shared__ __attribute__((aligned(16))) uint4 Wl[R::W_VECS];
  __shared__ __attribute__((aligned(16))) uint4 Ah[2][A_VECS];
  // per GEMM column: bias, weight scale, fp8 output scale
  __shared__ __attribute__((aligned(16))) float prm[3 * BN];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lrow = lane & 31, lhalf = lane >> 5;
  const int merged = a.transposed == 2;
  const int rc = a.K_pad * (int)sizeof(T) / 16, rcp = rc + 1;
  const int n_slices = a.cin_pad / BK;

  // Per-phase launches: workgroup b serves phase (b / 8) % 4 (so every XCD
  // has all four), with the remaining bits numbering it within its phase.
  int G = gridDim.x, b = blockIdx.x, phase = 0;
  if constexpr (TAPS == 4) {
    if (G % 32 == 0) {
      phase = (b >> 3) & 3;
      b = (b & 7) | ((b >> 5) << 3);
    } else {
      phase = b & 3;
      b >>= 2;
    }
    G >>= 2;
  }
  const int pyph = phase >> 1, pxph = phase & 1;
  // This workgroup's blocks: each XCD (workgroups round-robin over 8) owns a
  // contiguous range of blocks, so neighbouring blocks' shared halo rows
  // meet in its L2; its workgroups take the range's blocks in turn.
  int t_first = b, t_step = G, t_end = n_tiles;
  if (G % 8 == 0) {
    const int x = b & 7, q = n_tiles >> 3, r = n_tiles & 7;
    const int base = x * q + min(x, r);
    t_first = base + (b >> 3);
    t_step = G >> 3;
    t_end = base + q + (x < r ? 1 : 0);
  }
  const int tiles_x = (a.Wo + TW - 1) / TW, tiles_y = (a.Ho + TH - 1) / TH;
  const int per_img = tiles_x * tiles_y;

  const T* in = reinterpret_cast<const T*>(a.in);
  const T* wgt = reinterpret_cast<const T*>(a.wgt) + (long)phase * a.cout_pad * a.K_pad;
  const T* zero = reinterpret_cast<const T*>(a.zero);

  // The per-column parameters, once per workgroup (the pipeline's first
  // barrier publishes them): column n of a phase-merged conv is output
  // channel n % cout of phase n / cout.
  const int cout_m = merged ? a.cout : 1;
  if (tid < BN) {
    const bool ok = tid < a.n_rows;
    const int o = ok ? (merged ? tid % cout_m : tid) : 0;
    prm[tid] = ok ? a.bias[o] : 0.f;
    prm[BN + tid] = ok && a.w_scale ? a.w_scale[o] : 1.f;
    prm[2 * BN + tid] = ok && a.out_scale ? a.out_scale[o] : 1.f;
  }

  // resident weights: slot v = (row v / rcp, chunk v % rcp); the pitch's
  // last chunk is never written or read
  for (int v0 = 0; v0 < BN * rcp; v0 += NT) {
    const int v = v0 + tid;
    const int row = v / rcp, c = v - row * rcp;
    if (v < BN * rcp && c < rc) load_to_lds(wgt + (long)row * a.K_pad + c * VEC, &Wl[v0 + wave * 64]);
  }

  // halo slot tid + i*NT = (halo row, physical chunk tid % CH): its place in
  // the 18x18 halo and the channel offset of the chunk stored there
  const int chunk = tid % CH;
  int h_y[A_IT], h_x[A_IT], h_c[A_IT];
#pragma unroll
  for (int i = 0; i < A_IT; ++i) {
    const int hrow = (tid + i * NT) / CH;
    h_y[i] = hrow / HW;
    h_x[i] = hrow % HW;
    h_c[i] = (chunk ^ Halo::key(hrow)) * VEC;
  }
  auto issue_halo = [&](int t, int s, int buf) {
    const int img = t / per_img, rem = t - img * per_img;
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
    const T* src0 = in + (long)img * a.in_img_stride + s * BK;
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const int iy = ty0 - 1 + h_y[i], ix = tx0 - 1 + h_x[i];
      const bool ok = tid + i * NT < A_VECS && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
      const T* src = ok ? src0 + ((iy * a.Wi + ix) * a.in_ld + h_c[i]) : zero;
      if (A_VECS % NT == 0 || tid + i * NT < A_VECS) load_to_lds(src, &Ah[buf][i * NT + wave * 64]);
    }
  };

  // this lane's output pixel (A fragment row) in the block
  const int prow = wave * 32 + lrow;
  const int py = prow / TW, pxx = prow % TW;
  f32x16 acc[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;

  // A tap's fragments (this lane half's CH/2 chunks of the pixel, and of
  // each weight row) are read into one register set while the MFMAs of the
  // previous tap consume the other, so LDS latency is not paid per MFMA.
  constexpr int QN = CH / 2;
  auto load_tap = [&](int buf, int s, int tap, uint4 (&fa)[QN], uint4 (&fb)[FN][QN]) {
    // (y + dy + 1, x + dx + 1): the 3x3 neighbourhood, or the 2x2 taps of
    // the phase, dy = py - tap / 2, dx = px - tap % 2
    const int hidx = TAPS == 9 ? (py + tap / 3) * HW + pxx + tap % 3
                               : (py + pyph - (tap >> 1) + 1) * HW + pxx + pxph - (tap & 1) + 1;
    const int kc = (s * TAPS + tap) * CH + lhalf * QN;  // (slice, tap) chunk in a weight row
#pragma unroll
    for (int q = 0; q < QN; ++q) fa[q] = Ah[buf][Halo::swz(hidx, lhalf * QN + q)];
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int q = 0; q < QN; ++q) fb[f][q] = Wl[(f * 32 + lrow) * rcp + kc + q];
  };
  auto mma_tap = [&](const uint4 (&fa)[QN], const uint4 (&fb)[FN][QN]) {
    if constexpr (sizeof(T) == 1) {
#pragma unroll
      for (int q = 0; q < QN; q += 2)
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          if constexpr (SW)
            mfma_f8(acc[f], fb[f][q], fb[f][q + 1], fa[q], fa[q + 1]);
          else
            mfma_f8(acc[f], fa[q], fa[q + 1], fb[f][q], fb[f][q + 1]);
        }
    } else {
#pragma unroll
      for (int q = 0; q < QN; ++q)
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          if constexpr (SW)
            mfma_chunk<T>(acc[f], fb[f][q], fa[q]);
          else
            mfma_chunk<T>(acc[f], fa[q], fb[f][q]);
        }
    }
  };
  auto compute = [&](int buf, int s) {
    uint4 fa[2][QN], fb[2][FN][QN];
    load_tap(buf, s, 0, fa[0], fb[0]);
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap) {
      if (tap + 1 < TAPS) load_tap(buf, s, tap + 1, fa[(tap + 1) & 1], fb[(tap + 1) & 1]);
      // keep the next tap's reads ahead of this tap's MFMAs (the scheduler
      // would otherwise sink each read to its MFMA)
      __builtin_amdgcn_sched_barrier(0);
      mma_tap(fa[tap & 1], fb[tap & 1]);
    }
  };

  // Epilogue of block t, whose last slice was computed from halo buffer buf.
  // output pixel of GEMM grid point (oy, ox) when not phase-merged
  auto out_pix = [&](int oy, int ox) {
    return TAPS == 4 ? (long)(2 * oy + pyph) * a.Wout + 2 * ox + pxph : (long)oy * a.Wout + ox;
  };
  auto epilogue_staged = [&](int t, int buf) {
    // lane l holds, for fragment f, pixel wave*32 + l%32 and GEMM columns
    // f*32 + 8g + 4*(l/32) + q (g, q = 0..3). Bias, scale and ReLU in
    // registers; the wave's 32 x BN tile goes to its own part of the halo
    // buffer every wave has now finished with (rows of BN values, 16-byte
    // chunks XOR-swizzled by row), and is read back as 16-byte chunks.
    const int img = t / per_img, rem = t - img * per_img;
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
    const int E = a.out_scale ? 1 : 2;  // output element bytes (fp8 or bf16)
    const int pitch = BN * E, cpr = pitch / 16;
    char* region = reinterpret_cast<char*>(&Ah[buf][0]) + wave * 32 * pitch;
    __syncthreads();
    // specialised on the uniform flags (ReLU, output type, calibration's
    // running |max|): no per-value branch
    auto convert = [&](auto relu_c, auto e_c, auto amax_c) {
      constexpr bool RELU = decltype(relu_c)::value, AMAX = decltype(amax_c)::value;
      constexpr int EE = decltype(e_c)::value;
      constexpr int PITCH = BN * EE, CPR = PITCH / 16;
      char* rg = reinterpret_cast<char*>(&Ah[buf][0]) + wave * 32 * PITCH;
      const float* pr = prm;
#pragma unroll
      for (int f = 0; f < FN; ++f) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int n = f * 32 + 8 * g + 4 * lhalf;  // first of 4 GEMM columns (one output phase)
          const float4 b4 = *reinterpret_cast<const float4*>(pr + n);
          const float4 s4 = *reinterpret_cast<const float4*>(pr + BN + n);
          const float bq[4] = {b4.x, b4.y, b4.z, b4.w}, sq[4] = {s4.x, s4.y, s4.z, s4.w};
          float v[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float x = acc[f][4 * g + q] * sq[q] + bq[q];
            if constexpr (RELU) x = fmaxf(x, 0.f);
            v[q] = x;
          }
          if constexpr (AMAX) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (n + q < a.n_rows) {
                const int o = merged ? (n + q) % cout_m : n + q;
                atomicMax(reinterpret_cast<unsigned*>(a.amax) + o, __float_as_uint(fabsf(v[q])));
              }
          }
          const int byte = n * EE;
          char* dst = rg + lrow * PITCH + (((byte >> 4) ^ (lrow & (CPR - 1))) << 4) + (byte & 15);
          if constexpr (EE == 2) {
            uint2 w;
            w.x = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[0], v[1]}, bf16x2));
            w.y = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[2], v[3]}, bf16x2));
            *reinterpret_cast<uint2*>(dst) = w;
          } else {
            const float4 o4 = *reinterpret_cast<const float4*>(pr + 2 * BN + n);
            const float os[4] = {o4.x, o4.y, o4.z, o4.w};
            uint32_t w = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) w |= (uint32_t)to_f8(v[q] * os[q]) << (8 * q);
            *reinterpret_cast<uint32_t*>(dst) = w;
          }
        }
      }
    };
    using F0 = std::false_type;
    using F1 = std::true_type;
    using E1 = std::integral_constant<int, 1>;
    using E2 = std::integral_constant<int, 2>;
    if (a.amax) {
      if (E == 2) {
        if (a.relu) convert(F1{}, E2{}, F1{});
        else convert(F0{}, E2{}, F1{});
      } else {
        if (a.relu) convert(F1{}, E1{}, F1{});
        else convert(F0{}, E1{}, F1{});
      }
    } else if (E == 2) {
      if (a.relu) convert(F1{}, E2{}, F0{});
      else convert(F0{}, E2{}, F0{});
    } else {
      if (a.relu) convert(F1{}, E1{}, F0{});
      else convert(F0{}, E1{}, F0{});
    }
    // the wave reads back only its own region: its LDS operations complete
    // in order, so waiting for them is enough
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    const int run = 16 / E;
    for (int q = lane; q < 32 * cpr; q += 64) {
      const int p = q / cpr, ch = q - p * cpr;
      const int row = wave * 32 + p;
      int oy = ty0 + row / TW, ox = tx0 + row % TW;
      const int n = ch * run;
      if (oy >= a.Ho || ox >= a.Wo || n >= a.n_rows) continue;
      long off;
      if (!merged) {
        off = out_pix(oy, ox) * a.out_ld + n;
      } else {
        const int ph = n / cout_m, o = n - ph * cout_m;
        off = ((long)(2 * oy + (ph >> 1)) * a.Wout + 2 * ox + (ph & 1)) * a.out_ld + o;
      }
      const uint4 w = *reinterpret_cast<const uint4*>(region + p * pitch + ((ch ^ (p & (cpr - 1))) << 4));
      *reinterpret_cast<uint4*>(reinterpret_cast<char*>(a.out) + ((long)img * a.out_img_stride + off) * E) = w;
    }
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;
  };
  auto epilogue_f32 = [&](int t, int buf) {
    // as epilogue_staged, with float values: row p of the wave's region
    // holds the BN GEMM columns of pixel p; then one lane per output pixel
    // (four per GEMM pixel when phase-merged) gathers its cout values and
    // writes (or adds) them with float4 accesses where they allow.
    const int img = t / per_img, rem = t - img * per_img;
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
    constexpr int CPR = BN * 4 / 16;  // 16-byte chunks per staged row
    float* region = reinterpret_cast<float*>(reinterpret_cast<char*>(&Ah[buf][0]) + wave * 32 * BN * 4);
    const float* pr = prm;
    __syncthreads();
#pragma unroll
    for (int f = 0; f < FN; ++f) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int n0 = f * 32 + 8 * g + 4 * lhalf;
        const float4 b4 = *reinterpret_cast<const float4*>(pr + n0);
        const float4 s4 = *reinterpret_cast<const float4*>(pr + BN + n0);
        const float bq[4] = {b4.x, b4.y, b4.z, b4.w}, sq[4] = {s4.x, s4.y, s4.z, s4.w};
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int n = n0 + q;
          float x = acc[f][4 * g + q] * sq[q] + bq[q];
          if (a.relu) x = fmaxf(x, 0.f);
          if (a.amax && n < a.n_rows)
            atomicMax(reinterpret_cast<unsigned*>(a.amax) + (merged ? n % cout_m : n), __float_as_uint(fabsf(x)));
          v[q] = x;
        }
        *reinterpret_cast<float4*>(region + lrow * BN + (((n0 >> 2) ^ (lrow & (CPR - 1))) << 2)) =
            make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // own region only: in-order LDS suffices
    __builtin_amdgcn_wave_barrier();
    const int nph = merged ? 4 : 1;
    const int per = merged ? cout_m : a.cout;  // values per output pixel
    for (int q = lane; q < 32 * nph; q += 64) {
      const int p = q / nph, ph = q - p * nph;
      const int row = wave * 32 + p;
      const int oy = ty0 + row / TW, ox = tx0 + row % TW;
      if (oy >= a.Ho || ox >= a.Wo) continue;
      const long pix = merged ? (long)(2 * oy + (ph >> 1)) * a.Wout + 2 * ox + (ph & 1) : out_pix(oy, ox);
      float* dst = reinterpret_cast<float*>(a.out) + (long)img * a.out_img_stride + pix * a.out_ld;
      for (int c0 = 0; c0 < per; c0 += 4) {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int col = ph * per + c0 + k;
          v[k] = (c0 + k < per) ? region[p * BN + (((col >> 2) ^ (p & (CPR - 1))) << 2) + (col & 3)] : 0.f;
        }
        if (c0 + 4 <= per) {
          float4 w = make_float4(v[0], v[1], v[2], v[3]);
          if (a.accumulate) {
            const float4 old = *reinterpret_cast<const float4*>(dst + c0);
            w.x += old.x;
            w.y += old.y;
            w.z += old.z;
            w.w += old.w;
          }
          *reinterpret_cast<float4*>(dst + c0) = w;
        } else {
          for (int k = 0; c0 + k < per; ++k) dst[c0 + k] = a.accumulate ? dst[c0 + k] + v[k] : v[k];
        }
      }
    }
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;
  };
  // (pixels as A): lane l holds channel f*32 + l%32 of 16 pixels per
  // fragment; registers straight to global memory.
  auto epilogue = [&](int t) {
    const int img = t / per_img, rem = t - img * per_img;
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int n = f * 32 + lrow;
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
      if (!n_ok) continue;
      const float* pr = prm;
      const float bn = pr[n];
      const float ws = pr[BN + n];
      float amax = 0.f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wave * 32 + (e >> 2) * 8 + lhalf * 4 + (e & 3);
        const int oy = ty0 + row / TW, ox = tx0 + row % TW;
        if (oy >= a.Ho || ox >= a.Wo) continue;
        // merged: the GEMM grid point's phase-(0, 0) output
        const long pix = merged ? (long)(2 * oy) * a.Wout + 2 * ox : out_pix(oy, ox);
        float v = acc[f][e] * ws + bn;
        if (a.relu) v = fmaxf(v, 0.f);
        amax = fmaxf(amax, fabsf(v));
        store_out<T>(a, (long)img * a.out_img_stride + pix * a.out_ld + col, o, v);
      }
      if (a.amax) atomicMax(reinterpret_cast<unsigned*>(a.amax) + o, __float_as_uint(amax));
    }
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;
  };

  // one pipeline of (block, slice) steps; step j computes from halo buffer
  // j & 1 while the next step's halo loads into the other one. The first
  // wait also covers the resident weights.
  // The issue cursor (it, is) runs one step ahead of the computed step; a
  // single call site keeps the loop body small.
  int it = t_first, is = 0;
  auto advance = [&]() {
    if (++is == n_slices) {
      is = 0;
      it += t_step;
    }
  };
  if (it < t_end && n_slices > 0) issue_halo(it, is, 0);
  advance();
  int j = 0;
  for (int t = t_first; t < t_end; t += t_step) {
    for (int s = 0; s < n_slices; ++s, ++j) {
      wait_vm<0>();
      __syncthreads();
      if (it < t_end) issue_halo(it, is, (j + 1) & 1);
      advance();
      compute(j & 1, s);
    }
    if constexpr (EPI == 1)
      epilogue_staged(t, (j - 1) & 1);
    else if constexpr (EPI == 2)
      epilogue_f32(t, (j - 1) & 1);
    else
      epilogue(t);
  }
  wait_vm<0>();  // nothing outstanding when the workgroup ends
}

// Compute units of the current device (the persistent grid's size).
inline int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 8;
  }
  return cus;
}

template <typename T, int BN, int TAPS>
hipError_t launch_resident_epi(const ConvArgs& a, hipStream_t s, int grid, long tiles, bool staged16,
                               bool staged32) {
  if constexpr (sizeof(T) != 4) {
    if (staged16) {
      hipLaunchKernelGGL((conv_resident<T, BN, 1, TAPS>), dim3(grid), dim3(Resident::NT), 0, s, a, (int)tiles);
      return hipGetLastError();
    }
  }
  if constexpr (BN == 32) {
    if (staged32) {
      hipLaunchKernelGGL((conv_resident<T, BN, 2, TAPS>), dim3(grid), dim3(Resident::NT), 0, s, a, (int)tiles);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((conv_resident<T, BN, 0, TAPS>), dim3(grid), dim3(Resident::NT), 0, s, a, (int)tiles);
  return hipGetLastError();
}

template <typename T, int BN>
hipError_t launch_resident(const ConvArgs& a, hipStream_t s) {
  constexpr int VEC = 16 / (int)sizeof(T);
  if (!resident_ok(a, BN, (int)sizeof(T)) || a.n_rows <= 0 || a.in_ld % VEC != 0 || a.in_ld < a.cin_pad)
    return hipErrorInvalidValue;
  if ((long)a.Hi * a.Wi * a.in_ld >= (1L << 31)) return hipErrorInvalidValue;
  const long tiles = (long)a.n_img * ((a.Ho + Resident::TH - 1) / Resident::TH) *
                     ((a.Wo + Resident::TW - 1) / Resident::TW);
  if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
  const int cus = device_cus();
  const long per_dev = cus >= 8 ? cus / 8 * 8 : cus;  // one workgroup per compute unit
  // per-phase launches: a multiple of 4 workgroups, a quarter per phase
  const long want = a.transposed == 1 ? 4 * tiles : tiles;
  const int grid = a.transposed == 1 ? (int)(want < per_dev ? want : per_dev / 4 * 4)
                                     : (int)(want < per_dev ? want : per_dev);
  if (grid <= 0) return hipErrorInvalidValue;
  // staged epilogues: bf16/fp8 outputs in 16-byte channel runs, or float
  // outputs of a 32-column tile in 16-byte aligned pixels
  const int run = a.out_scale ? 16 : 8;
  const bool out16 = ((uintptr_t)a.out & 15) == 0;
  const bool staged16 = sizeof(T) != 4 && !a.out_f32 && a.cout % run == 0 && a.out_ld % run == 0 &&
                        a.out_img_stride % run == 0 && out16;
  const bool staged32 = BN == 32 && a.out_f32 && a.out_ld % 4 == 0 && a.out_img_stride % 4 == 0 && out16;
  if (a.transposed == 1) return launch_resident_epi<T, BN, 4>(a, s, grid, tiles, staged16, staged32);
  return launch_resident_epi<T, BN, 9>(a, s, grid, tiles, staged16, staged32);
}

}  // namespace convk
}  // namespace ffv
