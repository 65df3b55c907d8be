// Network executor: weights, packed per precision; workspace planning; the
// forward launch sequence of the view-interpolation network.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace ffv {

struct Status {
  int code = 0;  // ffv_status value
  std::string msg;
  static Status ok() { return Status(); }
  static Status err(int c, const std::string& m) {
    Status s;
    s.code = c;
    s.msg = m;
    return s;
  }
  bool good() const { return code == 0; }
};

// One convolution layer as stored in the weights file, and packed on device.
struct Layer {
  std::string name;
  bool transposed = false;
  int cin = 0, cout = 0, stride = 1;
  int cin_pad = 0, K = 0, K_pad = 0, cout_pad = 0;
  int mode = 0;  // ConvArgs::transposed: 0 conv, 1 per-phase transposed, 2 phase-merged
  ConvTile tile = ConvTile::N256;
  std::vector<float> w_host;  // file layout
  std::vector<float> b_host;
  void* w_dev = nullptr;      // packed [phase][cout_pad][K_pad], activation dtype
  float* b_dev = nullptr;
};

struct WeightsFile {
  int base_width = 0;
  bool t_plane = true;
  std::map<std::string, Layer> layers;
};

Status read_weights_file(const std::string& path, WeightsFile& out);

// Tile and padding choice for a layer (shared by the net and the op entry).
void plan_layer(Layer& L);
// Pack L.w_host for dtype dt into a host byte buffer laid out as the conv
// kernel reads it.
std::vector<uint8_t> pack_layer(const Layer& L, DType dt);

struct KernelStat {
  long launches = 0;
  double ms = 0.0;
  double work = 0.0;
};

class Net {
 public:
  Net() = default;
  ~Net();
  Status init(const std::string& weights_path, int precision, int device, hipStream_t stream,
              size_t workspace_cap);
  Status interpolate(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                     const float* t, int n_t, float* out);
  Status debug_tap(const std::string& name, float* dst, size_t cap, int dims[3]);
  void set_debug(bool on) { debug_ = on; }
  void set_profiling(bool on);
  Status kernel_stats(const std::string& name, long* launches, double* ms, double* work);
  DType dtype() const { return dt_; }
  int device() const { return device_; }
  hipStream_t stream() const { return stream_; }

 private:
  struct Geo {
    int H = 0, W = 0, Hp = 0, Wp = 0;
    long P = 0;
  };
  // Byte offsets of every buffer in the workspace for one geometry.
  struct Plan {
    Geo g;
    int n_cam = 0, n_view = 0;
    size_t total = 0;
    // camera region
    size_t X4, Xa, L0, L1, ctx[4], ctmp;
    // view region
    size_t FM[3], I2, Fp[4], views;
    // aliased phase region
    size_t xin, a1, bA, bB;                          // VIBlocks
    size_t x0u, lvl[4], etmp, u4;                    // U-Net
  };

  Status make_plan(const Geo& g, int n_cam, int n_view, Plan& p) const;
  Status ensure_workspace(size_t bytes);
  Status run_chunk(const Plan& p, const ViewDesc* views_host, int n_view, float* const* outs);
  Status conv(const Layer& L, const void* in, int in_ld, long in_img_stride, int Hi, int Wi,
              int n_img, void* out, int out_ld, long out_img_stride, bool out_f32, bool accumulate,
              bool relu);
  const Layer& layer(const std::string& n) const { return layers_.at(n); }
  char* ws(size_t off) const { return static_cast<char*>(ws_) + off; }
  void prof_begin();
  void prof_end(const char* cls, double work);
  Status check(hipError_t e, const char* what);

  std::map<std::string, Layer> layers_;
  int base_width_ = 32;
  bool t_plane_ = true;
  DType dt_ = DType::F32;
  int device_ = 0;
  hipStream_t stream_ = nullptr;
  bool own_stream_ = false;
  size_t ws_cap_ = 0;
  void* ws_ = nullptr;
  size_t ws_bytes_ = 0;
  void* src_ptrs_ = nullptr;  // device array of camera image pointers
  size_t src_ptrs_cap_ = 0;
  bool debug_ = false;
  bool have_taps_ = false;
  Plan last_plan_{};

  bool profiling_ = false;
  struct PendingEvt {
    hipEvent_t a, b;
    std::string cls;
    double work;
  };
  std::vector<PendingEvt> pending_;
  std::vector<hipEvent_t> evt_pool_;
  hipEvent_t cur_start_ = nullptr;
  std::map<std::string, KernelStat> stats_;
};

}  // namespace ffv
