// Instantiations of the implicit-GEMM convolution kernel (conv_kernel.h)
// used by the library, one per N-tile class, and of the halo-reuse kernel
// (conv_halo.h). All use 128-byte K steps (conv_k_step), which the weight
// packing's K order depends on.
#include "conv_halo.h"
#include "conv_kernel.h"
#include "conv_resident.h"
#include "conv_resident_s2.h"

namespace ffv {

namespace {

// the few-channel resident kernel for the (channel chunks, N tile, stride)
// triples whose buffers fit LDS
template <typename T, int PC, int BN, int ST>
hipError_t launch_s2_pc(const ConvArgs& a, hipStream_t s) {
  if constexpr (convk::ResS2::vecs(PC, BN, ST) <= convk::ResS2::LDS_VECS)
    return convk::launch_resident_s2<T, PC, BN, ST>(a, s);
  else
    return hipErrorInvalidValue;
}

template <typename T, int BN, int ST>
hipError_t launch_s2_st(const ConvArgs& a, hipStream_t s) {
  if (a.cin_pad % 8 != 0) return hipErrorInvalidValue;
  switch (a.cin_pad / 8) {
    case 1: return launch_s2_pc<T, 1, BN, ST>(a, s);
    case 2: return launch_s2_pc<T, 2, BN, ST>(a, s);
    case 3: return launch_s2_pc<T, 3, BN, ST>(a, s);
    case 4: return launch_s2_pc<T, 4, BN, ST>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int BN>
hipError_t launch_s2(const ConvArgs& a, hipStream_t s) {
  return a.stride == 1 ? launch_s2_st<T, BN, 1>(a, s) : launch_s2_st<T, BN, 2>(a, s);
}

template <typename T>
hipError_t launch_t(ConvTile tile, const ConvArgs* g, int n, hipStream_t s) {
  using namespace convk;
  // the persistent kernels take one image group
  if (!conv_tile_groupable(tile) && n != 1) return hipErrorInvalidValue;
  switch (tile) {
    case ConvTile::N256:
      return launch_variant<T, 256, 256, 4, 2, 128, 2, 1>(g, n, s);
    case ConvTile::N128:
      return launch_variant<T, 256, 128, 4, 2, 128, 2, 1>(g, n, s);
    case ConvTile::N64:
      return launch_variant<T, 256, 64, 8, 1, 128, 2, 1>(g, n, s);
    case ConvTile::N32:
      return launch_variant<T, 256, 32, 8, 1, 128, 2, 1>(g, n, s);
    case ConvTile::H32:
      return launch_halo<T>(g[0], s);
    case ConvTile::H256:
      return launch_variant<T, 256, 256, 4, 2, 128, 2, 1, true>(g, n, s);
    case ConvTile::H128:
      return launch_variant<T, 256, 128, 4, 2, 128, 2, 1, true>(g, n, s);
    case ConvTile::Q256:
      return launch_variant<T, 256, 256, 2, 4, 128, 2, 1, true>(g, n, s);
    case ConvTile::P256:
      return launch_variant<T, 256, 256, 4, 2, 128, 2, 1, true, true>(g, n, s);
    case ConvTile::R32:
      return launch_resident<T, 32>(g[0], s);
    case ConvTile::R64:
      return launch_resident<T, 64>(g[0], s);
    case ConvTile::S32:
      return launch_s2<T, 32>(g[0], s);
    case ConvTile::S64:
      return launch_s2<T, 64>(g[0], s);
    case ConvTile::S128:
      return launch_s2<T, 128>(g[0], s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int conv_k_step(DType dt) { return dt == DType::F32 ? 32 : (dt == DType::BF16 ? 64 : 128); }

bool conv_halo_tile_ok(DType dt, const ConvArgs& a) { return convk::halo_tile_ok(a, conv_k_step(dt)); }

bool conv_resident_ok(DType dt, const ConvArgs& a, int bn) {
  ConvArgs b = a;
  b.tile_w = convk::Resident::TW;
  return convk::resident_ok(b, bn, (int)dtype_size(dt));
}

bool conv_resident_s2_ok(DType dt, const ConvArgs& a, int bn) {
  using convk::ResS2;
  if (a.cin_pad % 8 != 0 || a.cin_pad < 8 || a.cin_pad > 32 || (a.stride != 1 && a.stride != 2)) return false;
  const int pc = a.cin_pad / 8, st = a.stride;
  if (bn != 32 && bn != 64 && bn != 128) return false;
  return ResS2::vecs(pc, bn, st) <= ResS2::LDS_VECS && convk::resident_s2_ok(a, pc, bn, st, (int)dtype_size(dt));
}

bool conv_halo_ok(DType dt, const ConvArgs& a) {
  ConvArgs b = a;
  b.tile_w = convk::Halo::TW;
  return convk::halo_ok(b, conv_k_step(dt));
}

int conv_tile_width(int Ho, int Wo) {
  int best = 16;
  long best_area = -1;
  for (int tw : {16, 32, 8, 64, 128, 256}) {
    const int th = 256 / tw;
    const long area = (long)((Ho + th - 1) / th) * th * ((Wo + tw - 1) / tw) * tw;
    if (best_area < 0 || area < best_area) {
      best_area = area;
      best = tw;
    }
  }
  return best;
}

hipError_t launch_conv_grouped(DType dt, ConvTile tile, const ConvArgs* g, int n, hipStream_t s) {
  if (n < 1 || n > ConvGroup::kMax) return hipErrorInvalidValue;
  // groups with no work are left out
  ConvArgs live[ConvGroup::kMax];
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (g[i].n_img > 0 && g[i].Ho > 0 && g[i].Wo > 0) live[m++] = g[i];
  if (m == 0) return hipSuccess;
  if (dt == DType::F32) return launch_t<float>(tile, live, m, s);
  if (dt == DType::FP8) return launch_t<f8>(tile, live, m, s);
  return launch_t<bf16>(tile, live, m, s);
}

hipError_t launch_conv(DType dt, ConvTile tile, const ConvArgs& a, hipStream_t s) {
  return launch_conv_grouped(dt, tile, &a, 1, s);
}

}  // namespace ffv
