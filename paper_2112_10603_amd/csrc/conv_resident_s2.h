// Persistent 3x3 convolution (stride 2, or 1) for layers with few input
// channels, with the weights resident in LDS (supplementary layer table:
// the first conv of each VIBlock, 8 or 24 input channels to 128, and the
// convs of the U-Net and context-feature levels with 8 to 32 input
// channels).
//
// The generic kernel gathers these layers' A tiles in 16-byte pieces (one
// tap's 8 channels of one input pixel per piece), so each input pixel is
// fetched about 2.25 times per M tile, and a tile's K (9 x channels) is only
// two to five 128-byte steps: it spends its time waiting on loads. Here a
// workgroup stays on its compute unit with the whole weight matrix in LDS
// and walks output blocks of TH x 16 pixels; per block it loads the input
// halo, (2 TH + 1) x 33 pixels at stride 2 or (TH + 2) x 18 at stride 1,
// with all their channels, once, and every tap of every K chunk reads from
// it. The next block's halo loads into the second buffer while the current
// one computes. At stride 2 halo columns are stored by parity (even input
// columns, then odd), so the 32 pixels of an MFMA fragment read consecutive
// halo pixels at any tap; the pixel pitch is an odd number of 16-byte
// chunks, which keeps 16 consecutive pixels in distinct bank groups. K runs tap-major, as the weights of these layers
// are packed: 16-byte chunk q of a K row holds channels 8 (q % PC) .. +7 of
// tap q / PC, PC = channels / 8.
#pragma once

#include <type_traits>

#include "conv_resident.h"

namespace ffv {
namespace convk {

struct ResS2 {
  static constexpr int NT = 512;    // 8 waves
  static constexpr int TW = 16;     // output block width
  static constexpr int HE = TW + 1;       // stored even columns (stride 2)
  static constexpr int LDS_VECS = 9984;   // 159,744 bytes
  static constexpr int hwd(int st) { return st == 2 ? 2 * TW + 1 : TW + 2; }  // halo width
  static constexpr int hh(int st, int th) { return st == 2 ? 2 * th + 1 : th + 2; }  // halo height
  // output block height for an N tile: 8 rows (4 fragments of 32 pixels
  // x 2 column groups) for 64/128 columns, 16 rows for 32
  static constexpr int th(int bn) { return bn >= 64 ? 8 : 16; }
  static constexpr int pp(int pc) { return pc | 1; }  // odd pixel pitch in chunks
  static constexpr int kpad(int pc) { return (72 * pc + 63) / 64 * 64; }
  // LDS vectors: two halos, the weights (row pitch one chunk longer than
  // the row), the output staging area (bf16 at most)
  static constexpr int vecs(int pc, int bn, int st) {
    return 2 * hh(st, th(bn)) * hwd(st) * pp(pc) + bn * (kpad(pc) / 8 + 1) + th(bn) * TW * bn * 2 / 16;
  }
};

// Whether the resident kernel at stride st with PC 16-byte chunks per input
// pixel (channels = 8 PC) and an N tile of bn columns covers a launch.
inline bool resident_s2_ok(const ConvArgs& a, int pc, int bn, int st, int elem_bytes) {
  return elem_bytes == 2 && a.transposed == 0 && a.stride == st && a.taps == 9 && a.cin_pad == 8 * pc &&
         a.K == 9 * a.cin_pad && a.K_pad == ResS2::kpad(pc) && a.n_rows <= bn && bn <= a.cout_pad &&
         a.Ho == (a.Hi - 1) / st + 1 && a.Wo == (a.Wi - 1) / st + 1 &&
         ResS2::vecs(pc, bn, st) <= ResS2::LDS_VECS;
}

template <typename T, int PC, int BN, int ST>
__global__ __launch_bounds__(ResS2::NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void conv_resident_s2(ConvArgs a, int n_tiles) {
  using R = ResS2;
  constexpr int NT = R::NT, TW = R::TW, HWD = R::hwd(ST), HE = R::HE;
  constexpr int TH = R::th(BN), PP = R::pp(PC), KP = R::kpad(PC);
  constexpr int RC = KP / 8, RCP = RC + 1;  // weight row chunks, pitch
  constexpr int NRD = KP / 16;              // MFMA rounds (two chunks each)
  constexpr int HV = R::hh(ST, TH) * HWD * PP;  // vectors per halo buffer
  constexpr int HIT = (HV + NT - 1) / NT;
  constexpr int PG = TH * TW / 32;          // pixel groups (fragments of 32 pixels)
  constexpr int CG = 8 / PG;                // column groups
  constexpr int WC = BN / CG;               // columns per wave
  constexpr int FN = WC / 32;
  static_assert(FN >= 1 && PG * CG == 8, "8 waves of 32-pixel fragments");
  static_assert(R::vecs(PC, BN, ST) <= R::LDS_VECS, "LDS");
  constexpr int KQ = 9 * PC;                // real K chunks

  __shared__ __attribute__((aligned(16))) uint4 smem[R::LDS_VECS];
  // per output channel: bias, weight scale, fp8 output scale
  __shared__ __attribute__((aligned(16))) float prm[3 * BN];
  uint4* Hb = smem;                         // two halo buffers
  uint4* Wl = smem + 2 * HV;                // resident weights
  char* St = reinterpret_cast<char*>(smem + 2 * HV + BN * RCP);  // output staging

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lrow = lane & 31, lhalf = lane >> 5;
  const int pg = wave % PG, cg = wave / PG;
  // the per-channel parameters, once per workgroup (published by the
  // pipeline's first barrier)
  for (int c = tid; c < BN; c += NT) {
    const bool ok = c < a.n_rows;
    prm[c] = ok ? a.bias[c] : 0.f;
    prm[BN + c] = ok && a.w_scale ? a.w_scale[c] : 1.f;
    prm[2 * BN + c] = ok && a.out_scale ? a.out_scale[c] : 1.f;
  }

  const int G = gridDim.x, b = blockIdx.x;
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
  const T* wgt = reinterpret_cast<const T*>(a.wgt);
  const T* zero = reinterpret_cast<const T*>(a.zero);

  // resident weights (slot v = row v / RCP, chunk v % RCP; the last chunk
  // of a row's pitch is never written or read)
  for (int v0 = 0; v0 < BN * RCP; v0 += NT) {
    const int v = v0 + tid;
    const int row = v / RCP, c = v - row * RCP;
    if (v < BN * RCP && c < RC) load_to_lds(wgt + (long)row * a.K_pad + c * 8, &Wl[v0 + wave * 64]);
  }

  // halo slot tid + i*NT = (stored pixel, chunk): its input row and column
  // offsets from the block's top-left input sample, and the chunk
  int h_yx[HIT], h_c[HIT];
#pragma unroll
  for (int i = 0; i < HIT; ++i) {
    const int v = tid + i * NT;
    const int hp = v / PP, c = v - hp * PP;
    const int hy = hp / HWD, sc = hp - hy * HWD;
    const int hx = ST == 1 ? sc : (sc < HE ? 2 * sc : 2 * (sc - HE) + 1);
    h_yx[i] = (hy << 8) | hx;
    h_c[i] = (v < HV && c < PC) ? c : -1;
  }
  auto issue_halo = [&](int t, int buf) {
    const int img = t / per_img, rem = t - img * per_img;
    const int iy0 = ST * ((rem / tiles_x) * TH) - 1, ix0 = ST * ((rem % tiles_x) * TW) - 1;
    const T* src0 = in + (long)img * a.in_img_stride;
#pragma unroll
    for (int i = 0; i < HIT; ++i) {
      const int iy = iy0 + (h_yx[i] >> 8), ix = ix0 + (h_yx[i] & 255);
      const bool ok = h_c[i] >= 0 && iy >= 0 && iy < a.Hi && ix >= 0 && ix < a.Wi;
      const T* src = ok ? src0 + ((iy * a.Wi + ix) * a.in_ld + h_c[i] * 8) : zero;
      if (HV % NT == 0 || tid + i * NT < HV) load_to_lds(src, &Hb[buf * HV + i * NT + wave * 64]);
    }
  };

  // this lane's pixel of its fragment, and its halo base (tap (-1, -1))
  const int p = pg * 32 + lrow;
  const int py = p / TW, px = p % TW;
  // halo row ST py + dy + 1; stored column: at stride 1, px + dx + 1; at
  // stride 2, dx = -1 -> px, 0 -> HE + px, +1 -> px + 1
  auto a_slot = [&](int q) {  // K chunk q < KQ
    const int tap = q / PC, c = q % PC;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int sc = ST == 1 ? px + dx + 1 : (dx == 0 ? HE + px : px + (dx > 0 ? 1 : 0));
    return ((ST * py + dy + 1) * HWD + sc) * PP + c;
  };
  f32x16 acc[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;

  // Round r pairs K chunks q0 (lane half 0) and q0 + 4 (lane half 1), with
  // q0 = 8 (r / 4) + r % 4: the pairing and order the generic kernel's
  // 128-byte steps use, so both give the same sums bit for bit. Chunks past
  // the real K are zero in the weights, and read as zero here.
  auto read_round = [&](int buf, int r, uint4& xa, uint4 (&xb)[FN]) {
    const int q0 = 8 * (r >> 2) + (r & 3), q1 = q0 + 4;
    const int s0 = q0 < KQ ? a_slot(q0) : 0, s1 = q1 < KQ ? a_slot(q1) : 0;
    const bool ok = lhalf ? q1 < KQ : q0 < KQ;
    const uint4 v = Hb[buf * HV + (lhalf ? s1 : s0)];
    xa = ok ? v : make_uint4(0u, 0u, 0u, 0u);
    const int wq = lhalf ? q1 : q0;
#pragma unroll
    for (int f = 0; f < FN; ++f) xb[f] = Wl[(cg * WC + f * 32 + lrow) * RCP + wq];
  };
  auto compute = [&](int buf) {
    uint4 fa[2], fb[2][FN];
    read_round(buf, 0, fa[0], fb[0]);
#pragma unroll
    for (int r = 0; r < NRD; ++r) {
      if (r + 1 < NRD) read_round(buf, r + 1, fa[(r + 1) & 1], fb[(r + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int f = 0; f < FN; ++f) mfma_chunk<T>(acc[f], fb[r & 1][f], fa[r & 1]);  // weights as A
    }
  };

  // Epilogue: lane l holds pixel l%32 of the wave's fragment and columns
  // cg*WC + f*32 + 8g + 4*(l/32) + q. The wave's 32 x WC tile goes to its
  // own staging region (rows of WC values, 16-byte chunks XOR-swizzled by
  // row) and leaves as 16-byte stores of whole channel runs.
  const int E = a.out_scale ? 1 : 2;
  const int pitch = WC * E, cpr = pitch / 16;
  char* region = St + wave * 32 * WC * 2;
  // The conversion reads the parameters from LDS and is specialised on the
  // uniform flags (ReLU, output type, calibration's running |max|), with no
  // per-value branch.
  auto convert = [&](auto relu_c, auto e_c, auto amax_c) {
    constexpr bool RELU = decltype(relu_c)::value, AMAX = decltype(amax_c)::value;
    constexpr int EE = decltype(e_c)::value;
    constexpr int PITCH = WC * EE, CPR = PITCH / 16;
    const float* pr = prm;
#pragma unroll
    for (int f = 0; f < FN; ++f) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int cw = f * 32 + 8 * g + 4 * lhalf;  // column within the wave's tile
        const int n = cg * WC + cw;
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
          if (n < a.n_rows)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              atomicMax(reinterpret_cast<unsigned*>(a.amax) + n + q, __float_as_uint(fabsf(v[q])));
        }
        const int byte = cw * EE;
        char* dst = region + lrow * PITCH + (((byte >> 4) ^ (lrow & (CPR - 1))) << 4) + (byte & 15);
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
  auto epilogue = [&](int t) {
    const int img = t / per_img, rem = t - img * per_img;
    const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
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
    __builtin_amdgcn_s_waitcnt(0xC07F);  // own region only: in-order LDS suffices
    __builtin_amdgcn_wave_barrier();
    const int run = 16 / E;
    for (int q = lane; q < 32 * cpr; q += 64) {
      const int pr = q / cpr, ch = q - pr * cpr;
      const int pix = pg * 32 + pr;
      const int oy = ty0 + pix / TW, ox = tx0 + pix % TW;
      const int n = cg * WC + ch * run;
      if (oy >= a.Ho || ox >= a.Wo || n >= a.n_rows) continue;
      const long off = (long)img * a.out_img_stride + ((long)oy * a.Wout + ox) * a.out_ld + n;
      const uint4 w = *reinterpret_cast<const uint4*>(region + pr * pitch + ((ch ^ (pr & (cpr - 1))) << 4));
      *reinterpret_cast<uint4*>(reinterpret_cast<char*>(a.out) + off * E) = w;
    }
#pragma unroll
    for (int f = 0; f < FN; ++f)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[f][e] = 0.f;
  };

  // one step per block: its halo was loaded during the previous block
  if (t_first < t_end) issue_halo(t_first, 0);
  int j = 0;
  for (int t = t_first; t < t_end; t += t_step, ++j) {
    wait_vm<0>();
    __syncthreads();
    if (t + t_step < t_end) issue_halo(t + t_step, (j + 1) & 1);
    compute(j & 1);
    epilogue(t);
  }
  wait_vm<0>();
}

template <typename T, int PC, int BN, int ST>
hipError_t launch_resident_s2(const ConvArgs& a, hipStream_t s) {
  if constexpr (sizeof(T) != 2) {
    return hipErrorInvalidValue;
  } else {
    if (!resident_s2_ok(a, PC, BN, ST, (int)sizeof(T)) || a.n_rows <= 0 || a.in_ld % 8 != 0 ||
        a.in_ld < a.cin_pad)
      return hipErrorInvalidValue;
    // the epilogue stages bf16/fp8 outputs in 16-byte channel runs
    const int run = a.out_scale ? 16 : 8;
    if (a.out_f32 || a.cout % run != 0 || a.out_ld % run != 0 || a.out_img_stride % run != 0 ||
        ((uintptr_t)a.out & 15) != 0)
      return hipErrorInvalidValue;
    if ((long)a.Hi * a.Wi * a.in_ld >= (1L << 31)) return hipErrorInvalidValue;
    constexpr int TH = ResS2::th(BN);
    const long tiles = (long)a.n_img * ((a.Ho + TH - 1) / TH) * ((a.Wo + ResS2::TW - 1) / ResS2::TW);
    if (tiles > 0x7fffffffL) return hipErrorInvalidValue;
    const int cus = device_cus();
    const long per_dev = cus >= 8 ? cus / 8 * 8 : cus;
    const int grid = (int)(tiles < per_dev ? tiles : per_dev);
    hipLaunchKernelGGL((conv_resident_s2<T, PC, BN, ST>), dim3(grid), dim3(ResS2::NT), 0, s, a, (int)tiles);
    return hipGetLastError();
  }
}

}  // namespace convk
}  // namespace ffv
