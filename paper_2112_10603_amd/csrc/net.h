// Network executor: weights, packed per precision; workspace planning; the
// forward launch sequence of the view-interpolation network; the serving
// scheduler.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "scheduler.h"
#include "status.h"

namespace ffv {

// One convolution layer as stored in the weights file, and packed on device.
struct Layer {
  std::string name;
  bool transposed = false;
  int cin = 0, cout = 0, stride = 1;
  int cin_pad = 0, K = 0, K_pad = 0, cout_pad = 0;
  int mode = 0;  // ConvArgs::transposed: 0 conv, 1 per-phase transposed, 2 phase-merged
  int rows = 0;  // GEMM N: cout, or 4 * cout phase-merged
  ConvTile tile = ConvTile::N256;  // default N tile (narrowest that covers rows)
  std::vector<float> w_host;  // file layout
  std::vector<float> b_host;
  void* w_dev = nullptr;      // packed [phase][cout_pad][K_pad], activation dtype
  float* b_dev = nullptr;
  // FP8 (VIBlock 128/256-channel layers): fp8 weights with the producer's
  // activation scales folded in, the per-output-channel dequant scale, the
  // output quantisation scale (1 / activation scale) and calibration amax.
  void* w8_dev = nullptr;
  float* w8_scale = nullptr;
  float* out_scale = nullptr;
  float* amax = nullptr;
  std::vector<float> act_scale;  // per output channel: |activation| max / 448
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

// Image geometry: real size and the size padded to a multiple of 16.
struct Geo {
  int H = 0, W = 0, Hp = 0, Wp = 0;
  long P = 0;
  static Geo of(int H, int W);
  bool operator==(const Geo& o) const { return H == o.H && W == o.W; }
};

// Views of one size in a batch of several sizes: views first .. first+n-1,
// padded full-resolution size Hp x Wp.
struct ViewGroup {
  int first = 0, n = 0, Hp = 0, Wp = 0;
};

// Where kernels run: a stream and the base of a workspace; for a batch of
// views of several sizes, its size groups (the plan is sized for the
// largest, plan_hp being its padded height).
struct Exec {
  hipStream_t s = nullptr;
  char* ws = nullptr;
  bool prof = false;
  bool capture = false;  // the stream is being captured into a graph
  const ViewGroup* groups = nullptr;
  int n_groups = 0;
  int plan_hp = 0;
  char* at(size_t off) const { return ws + off; }
};

// Byte offsets of one camera's resident data inside a camera block.
struct CamPlan {
  size_t X4, Xa, L0, L1, ctx[4];
  size_t bytes;  // one camera block
  size_t ctmp;   // scratch per camera while building (context convs)
};

// Byte offsets of one chunk of views inside a view workspace.
struct ViewPlan {
  Geo g;
  int n_view = 0;
  size_t FM[3], I2, Fp[4], views;
  size_t xin, a1, bA, bB;          // VIBlocks
  size_t x0u, lvl[4], etmp, u4;    // U-Net (aliases the VIBlock buffers)
  size_t total = 0;
};

class HipExecutor;

class Net {
 public:
  Net();
  ~Net();
  Status init(const std::string& weights_path, int precision, int device, hipStream_t stream,
              size_t workspace_cap);
  Status interpolate(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                     const float* t, int n_t, float* out);
  // The Eq. 1 blend alone (no context features, U-Net or residual: the
  // paper's "w/o Refine" variant), same arguments and layout.
  Status interpolate_blend(const float* const* left, const float* const* right, int n_pairs, int H,
                           int W, const float* t, int n_t, float* out);
  // Dense views by recursive midpoints: `levels` = n gives, per pair, the
  // 2^n - 1 views at t = k/2^n (k = 1 .. 2^n - 1) in out[pair][k - 1], each
  // the t = 1/2 synthesis of its two neighbours; one batched call per level.
  Status interpolate_recursive(const float* const* left, const float* const* right, int n_pairs,
                               int H, int W, int levels, float* out);
  Status debug_tap(const std::string& name, float* dst, size_t cap, int dims[3]);
  // FP8 nets: run one view in bf16, record the VIBlock activations' per-channel
  // ranges, then quantise those layers' weights (needed before use).
  Status calibrate(const float* left, const float* right, int H, int W, float t);
  bool ready() const { return !fp8_ || calibrated_; }
  void set_debug(bool on) { debug_ = on; }
  // Replay interpolate()'s launch sequence as one hipGraph per call shape.
  void set_graphs(bool on);
  void set_profiling(bool on);
  Status kernel_stats(const std::string& name, long* launches, double* ms, double* work);
  // Runs the call like interpolate(), then times every candidate tile shape
  // (N tile width, M-tile pixel block width) of each convolution launch of
  // that call and keeps the fastest for its (layer, precision, grid,
  // images); later calls of that shape use them. *n_tuned = launches tuned.
  Status autotune(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                  const float* t, int n_t, float* out, int* n_tuned);
  Status save_tuning(const std::string& path);
  Status load_tuning(const std::string& path, int* n_loaded);
  DType dtype() const { return dt_; }
  int device() const { return device_; }
  // Whether launch sequences may be captured into graphs and replayed, and
  // a counter that changes whenever captured graphs become stale (tile
  // tuning, FP8 quantisation, the workspace, the graph switch itself).
  bool graphs_enabled() const { return graphs_ && !calibrating_ && !recording_; }
  uint64_t graph_epoch() const { return graph_epoch_.load(std::memory_order_acquire); }
  hipStream_t stream() const { return stream_; }

  // serving
  Status start_serving(size_t budget, float tick_ms, int max_batch_views);
  Scheduler* server() { return sched_.get(); }
  // Device allocation through the fault hook (FFV_FAULT=alloc:N).
  Status dev_alloc(void** p, size_t bytes, const char* what) const;

  // building blocks (also used by the server)
  CamPlan cam_plan(const Geo& g) const;
  ViewPlan view_plan(const Geo& g, int n_view) const;
  // Build n_cam cameras' resident data: src is a device table of n_cam
  // planar [3][H][W] images; camera i's block starts at blocks[i] (host
  // array of device pointers). ctmp is scratch of n_cam * cp.ctmp bytes.
  Status build_cameras(const Exec& x, const Geo& g, const float* const* src_dev, int n_cam,
                       char* const* blocks, char* ctmp, bool context = true);
  // Run nv views. views_on_device: `views` is a device table that stays
  // valid until the work completes; otherwise a host array copied to the
  // plan's view slot on the stream.
  Status run_views(const Exec& x, const ViewPlan& p, const CamDev* cams_dev, const ViewDesc* views,
                   int nv, bool views_on_device = false, bool refine = true);
  CamDev cam_dev(const Geo& g, char* block) const;
  Status check(hipError_t e, const char* what) const;

 private:
  Status interpolate_locked(const float* const* left, const float* const* right, int n_pairs, int H,
                            int W, const float* t, int n_t, float* out);
  // One batched call: view i*n_t + j of pair i at t[j] is written to
  // outs[i*n_t + j] (planar [3][H][W] device pointers).
  Status run_call(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                  const float* t, int n_t, float* const* outs, bool refine);
  Status ensure_workspace(size_t bytes);
  void drop_graphs();
  Status conv(const Exec& x, const Layer& L, const void* in, int in_ld, long in_img_stride, int Hi,
              int Wi, int n_img, void* out, int out_ld, long out_img_stride, bool out_f32,
              bool accumulate, bool relu, bool in_fp8 = false, bool out_fp8 = false);
  bool vib_fp8() const { return fp8_ && calibrated_ && !calibrating_; }
  Status quantize_vib_layers();
  const Layer& layer(const std::string& n) const { return layers_.at(n); }
  void prof_begin(const Exec& x);
  void record_event(const Exec& x, hipEvent_t e);
  bool prof_error_ = false;  // an event-record node could not be added
  void prof_end(const Exec& x, const char* cls, double work);

  std::map<std::string, Layer> layers_;
  int base_width_ = 32;
  bool t_plane_ = true;
  DType dt_ = DType::F32;
  bool fp8_ = false;          // FP8 VIBlocks (activation dtype elsewhere: bf16)
  std::atomic<bool> calibrated_{false};  // read by submitting threads
  bool calibrating_ = false;
  int device_ = 0;
  hipStream_t stream_ = nullptr;
  bool own_stream_ = false;
  size_t ws_cap_ = 0;
  void* ws_ = nullptr;
  size_t ws_bytes_ = 0;
  void* zero_ = nullptr;      // 256 zero bytes read by convs for taps outside the image
  bool debug_ = false;
  bool have_taps_ = false;
  ViewPlan last_plan_{};
  char* last_views_ws_ = nullptr;
  char* last_cam_l_ = nullptr;  // camera blocks of view 0 of the last call
  char* last_cam_r_ = nullptr;
  std::mutex call_mu_;        // serialises interpolate() per net

  // A timed kernel class interval: events recorded before and after.
  struct PendingEvt {
    hipEvent_t a, b;
    std::string cls;
    double work;
  };
  // Instantiated graphs of interpolate(), by call shape. Every pointer the
  // kernels take is either the net's (weights, workspace) or read from the
  // device tables written before each replay, so a graph depends only on
  // the key. With profiling on, the graph holds event-record nodes around
  // each kernel class (its `prof` intervals, read after every replay).
  struct GraphKey {
    int H, W, n_cam, n_view, chunk;
    const void* ws;
    bool fp8, prof, refine;
    bool operator<(const GraphKey& o) const {
      return std::tie(H, W, n_cam, n_view, chunk, ws, fp8, prof, refine) <
             std::tie(o.H, o.W, o.n_cam, o.n_view, o.chunk, o.ws, o.fp8, o.prof, o.refine);
    }
  };
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    std::vector<PendingEvt> prof;
  };
  bool graphs_ = true;
  std::atomic<uint64_t> graph_epoch_{0};
  std::map<GraphKey, GraphEntry> graph_cache_;
  void add_stat(const PendingEvt& pe);

  // Tile choices found by autotune(), per conv launch shape.
  struct TuneKey {
    std::string layer;
    int fp8, Ho, Wo, n_img;
    bool operator<(const TuneKey& o) const {
      return std::tie(layer, fp8, Ho, Wo, n_img) < std::tie(o.layer, o.fp8, o.Ho, o.Wo, o.n_img);
    }
  };
  struct TuneVal {
    ConvTile tile;
    int tile_w;
  };
  std::map<TuneKey, TuneVal> tuned_;
  bool recording_ = false;  // conv() records its launches for autotune()
  struct TuneRec {
    TuneKey key;
    ConvArgs a;
    DType dt;
  };
  std::vector<TuneRec> recs_;

  bool profiling_ = false;
  std::vector<PendingEvt> pending_;
  std::vector<hipEvent_t> evt_pool_;
  hipEvent_t cur_start_ = nullptr;
  std::map<std::string, KernelStat> stats_;

  // serving: the scheduler is destroyed before its executor
  std::unique_ptr<HipExecutor> exec_;
  std::unique_ptr<Scheduler> sched_;
};



}  // namespace ffv
