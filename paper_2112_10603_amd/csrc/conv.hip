// Instantiations of the implicit-GEMM convolution kernel (conv_kernel.h)
// used by the library, one per N-tile class, and of the halo-reuse kernel
// (conv_halo.h). All use 128-byte K steps (conv_k_step), which the weight
// packing's K order depends on.
#include "conv_halo.h"
#include "conv_kernel.h"
#include "conv_resident.h"

namespace ffv {

namespace {

template <typename T>
hipError_t launch_t(ConvTile tile, const ConvArgs& a, hipStream_t s) {
  using namespace convk;
  switch (tile) {
    case ConvTile::N256:
      return launch_variant<T, 256, 256, 4, 2, 128, 2, 1>(a, s);
    case ConvTile::N128:
      return launch_variant<T, 256, 128, 4, 2, 128, 2, 1>(a, s);
    case ConvTile::N64:
      return launch_variant<T, 256, 64, 8, 1, 128, 2, 1>(a, s);
    case ConvTile::N32:
      return launch_variant<T, 256, 32, 8, 1, 128, 2, 1>(a, s);
    case ConvTile::H32:
      return launch_halo<T>(a, s);
    case ConvTile::H256:
      return launch_variant<T, 256, 256, 4, 2, 128, 2, 1, true>(a, s);
    case ConvTile::H128:
      return launch_variant<T, 256, 128, 4, 2, 128, 2, 1, true>(a, s);
    case ConvTile::R32:
      return launch_resident<T, 32>(a, s);
    case ConvTile::R64:
      return launch_resident<T, 64>(a, s);
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

hipError_t launch_conv(DType dt, ConvTile tile, const ConvArgs& a, hipStream_t s) {
  if (a.n_img <= 0 || a.Ho <= 0 || a.Wo <= 0) return hipSuccess;
  if (dt == DType::F32) return launch_t<float>(tile, a, s);
  if (dt == DType::FP8) return launch_t<f8>(tile, a, s);
  return launch_t<bf16>(tile, a, s);
}

}  // namespace ffv
