// extern "C" entry points of libffv.so (declared in include/ffv.h).
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/ffv.h"
#include "fault.h"
#include "lap.h"
#include "net.h"
#include "op_conv.h"

struct ffv_net {
  ffv::Net net;
};

namespace {

thread_local std::string g_last_error;

ffv_status fail(int code, const std::string& msg) {
  g_last_error = msg;
  return (ffv_status)code;
}

ffv_status from(const ffv::Status& s) {
  if (s.good()) {
    g_last_error.clear();
    return FFV_OK;
  }
  return fail(s.code, s.msg);
}

// Shared argument checks of ffv_interpolate and ffv_autotune.
ffv_status check_call(ffv_net* net, const ffv_pair* views, int32_t n_pairs, const float* t,
                      int32_t n_t, float* out) {
  if (!net || !views || !t || !out) return fail(FFV_ERR_ARG, "null argument");
  if (n_pairs <= 0 || n_t <= 0) return fail(FFV_ERR_ARG, "n_pairs and n_t must be positive");
  const int H = views[0].height, W = views[0].width;
  if (H < 2 || W < 2) return fail(FFV_ERR_ARG, "height and width must be >= 2");
  if ((long)H * W > (1L << 28)) return fail(FFV_ERR_ARG, "image too large");
  for (int i = 0; i < n_pairs; ++i) {
    if (!views[i].left || !views[i].right) return fail(FFV_ERR_ARG, "null image pointer");
    if (views[i].height != H || views[i].width != W)
      return fail(FFV_ERR_ARG, "all pairs of one call must share height and width");
  }
  for (int j = 0; j < n_t; ++j)
    if (!(t[j] >= 0.f && t[j] <= 1.f)) return fail(FFV_ERR_ARG, "t must lie in [0, 1]");
  return FFV_OK;
}

}  // namespace

extern "C" {

void ffv_default_opts(ffv_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->abi_version = FFV_ABI_VERSION;
  o->precision = FFV_FP32;
  o->device = 0;
  o->graphs = 1;
  o->stream = nullptr;
  o->workspace_bytes = 0;
  o->hbm_budget_bytes = 0;
  o->tick_ms = 5.0f;
  o->max_batch_views = 0;
}

ffv_status ffv_create_net(const char* weights_path, const ffv_opts* opts, ffv_net** out) {
  if (!weights_path || !opts || !out) return fail(FFV_ERR_ARG, "null argument");
  *out = nullptr;
  if (opts->abi_version != FFV_ABI_VERSION) return fail(FFV_ERR_ARG, "ABI version mismatch");
  if (opts->precision != FFV_FP32 && opts->precision != FFV_BF16 &&
      opts->precision != FFV_FP8_E4M3)
    return fail(FFV_ERR_ARG, "unknown precision");
  try {
    ffv_net* n = new ffv_net();
    ffv::Status s = n->net.init(weights_path, opts->precision, opts->device,
                                (hipStream_t)opts->stream, opts->workspace_bytes);
    if (s.good()) n->net.set_graphs(opts->graphs != 0);
    if (s.good() && opts->hbm_budget_bytes > 0)
      s = n->net.start_serving(opts->hbm_budget_bytes, opts->tick_ms, opts->max_batch_views);
    if (!s.good()) {
      delete n;
      return from(s);
    }
    *out = n;
    g_last_error.clear();
    return FFV_OK;
  } catch (const std::bad_alloc&) {
    return fail(FFV_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

void ffv_destroy_net(ffv_net* net) { delete net; }

ffv_status ffv_autotune(ffv_net* net, const ffv_pair* views, int32_t n_pairs, const float* t,
                        int32_t n_t, float* out, int32_t* n_tuned) {
  const ffv_status c = check_call(net, views, n_pairs, t, n_t, out);
  if (c != FFV_OK) return c;
  try {
    std::vector<const float*> l(n_pairs), r(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
      l[i] = views[i].left;
      r[i] = views[i].right;
    }
    int n = 0;
    const ffv_status st = from(net->net.autotune(l.data(), r.data(), n_pairs, views[0].height,
                                                 views[0].width, t, n_t, out, &n));
    if (n_tuned) *n_tuned = n;
    return st;
  } catch (const std::bad_alloc&) {
    return fail(FFV_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_save_tuning(ffv_net* net, const char* path) {
  if (!net || !path) return fail(FFV_ERR_ARG, "null argument");
  try {
    return from(net->net.save_tuning(path));
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_load_tuning(ffv_net* net, const char* path, int32_t* n_loaded) {
  if (!net || !path) return fail(FFV_ERR_ARG, "null argument");
  try {
    int n = 0;
    const ffv_status st = from(net->net.load_tuning(path, &n));
    if (n_loaded) *n_loaded = n;
    return st;
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_interpolate_blend(ffv_net* net, const ffv_pair* views, int32_t n_pairs,
                                 const float* t, int32_t n_t, float* out) {
  const ffv_status c = check_call(net, views, n_pairs, t, n_t, out);
  if (c != FFV_OK) return c;
  try {
    std::vector<const float*> l(n_pairs), r(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
      l[i] = views[i].left;
      r[i] = views[i].right;
    }
    return from(net->net.interpolate_blend(l.data(), r.data(), n_pairs, views[0].height,
                                           views[0].width, t, n_t, out));
  } catch (const std::bad_alloc&) {
    return fail(FFV_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_interpolate_recursive(ffv_net* net, const ffv_pair* views, int32_t n_pairs,
                                     int32_t levels, float* out) {
  if (levels < 1 || levels > 10) return fail(FFV_ERR_ARG, "levels must lie in [1, 10]");
  const float half = 0.5f;
  const ffv_status c = check_call(net, views, n_pairs, &half, 1, out);
  if (c != FFV_OK) return c;
  try {
    std::vector<const float*> l(n_pairs), r(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
      l[i] = views[i].left;
      r[i] = views[i].right;
    }
    return from(net->net.interpolate_recursive(l.data(), r.data(), n_pairs, views[0].height,
                                               views[0].width, levels, out));
  } catch (const std::bad_alloc&) {
    return fail(FFV_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_interpolate(ffv_net* net, const ffv_pair* views, int32_t n_pairs, const float* t,
                           int32_t n_t, float* out) {
  const ffv_status c = check_call(net, views, n_pairs, t, n_t, out);
  if (c != FFV_OK) return c;
  const int H = views[0].height, W = views[0].width;
  if (n_pairs <= 0 || n_t <= 0) return fail(FFV_ERR_ARG, "n_pairs and n_t must be positive");
  try {
    std::vector<const float*> l(n_pairs), r(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
      l[i] = views[i].left;
      r[i] = views[i].right;
    }
    return from(net->net.interpolate(l.data(), r.data(), n_pairs, H, W, t, n_t, out));
  } catch (const std::bad_alloc&) {
    return fail(FFV_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

const char* ffv_last_error(void) { return g_last_error.c_str(); }

ffv_status ffv_calibrate(ffv_net* net, const ffv_pair* pair, float t) {
  if (!net || !pair || !pair->left || !pair->right) return fail(FFV_ERR_ARG, "null argument");
  if (pair->height < 2 || pair->width < 2) return fail(FFV_ERR_ARG, "height and width must be >= 2");
  if (!(t >= 0.f && t <= 1.f)) return fail(FFV_ERR_ARG, "t must lie in [0, 1]");
  try {
    return from(net->net.calibrate(pair->left, pair->right, pair->height, pair->width, t));
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_register_camera(ffv_net* net, int32_t cam_id, const float* image, int32_t height,
                               int32_t width) {
  if (!net || !image) return fail(FFV_ERR_ARG, "null argument");
  if (!net->net.server()) return fail(FFV_ERR_STATE, "serving is off (hbm_budget_bytes = 0)");
  try {
    return from(net->net.server()->register_camera(cam_id, image, height, width));
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_submit(ffv_net* net, const ffv_request* req, uint64_t* ticket) {
  if (!net || !req || !ticket) return fail(FFV_ERR_ARG, "null argument");
  if (!net->net.server()) return fail(FFV_ERR_STATE, "serving is off (hbm_budget_bytes = 0)");
  if (!net->net.ready()) return fail(FFV_ERR_STATE, "FP8 net needs ffv_calibrate first");
  ffv::Request r;
  r.cam_l = req->cam_left;
  r.cam_r = req->cam_right;
  r.t = req->t;
  r.out = req->out;
  r.tag = req->user_tag;
  try {
    return from(net->net.server()->submit(r, ticket));
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_submit_many(ffv_net* net, const ffv_request* reqs, int32_t n, uint64_t* tickets) {
  if (!net || n < 0 || (n > 0 && (!reqs || !tickets))) return fail(FFV_ERR_ARG, "null argument");
  if (!net->net.server()) return fail(FFV_ERR_STATE, "serving is off (hbm_budget_bytes = 0)");
  if (!net->net.ready()) return fail(FFV_ERR_STATE, "FP8 net needs ffv_calibrate first");
  std::vector<ffv::Request> rs(n);
  for (int i = 0; i < n; ++i) {
    rs[i].cam_l = reqs[i].cam_left;
    rs[i].cam_r = reqs[i].cam_right;
    rs[i].t = reqs[i].t;
    rs[i].out = reqs[i].out;
    rs[i].tag = reqs[i].user_tag;
  }
  try {
    int bad = -1;
    const ffv::Status st = net->net.server()->submit_many(rs.data(), n, tickets, &bad);
    if (!st.good() && bad >= 0) return fail(st.code, "request " + std::to_string(bad) + ": " + st.msg);
    return from(st);
  } catch (const std::exception& e) {
    return fail(FFV_ERR_DEVICE, e.what());
  }
}

ffv_status ffv_poll(ffv_net* net, uint64_t ticket, ffv_timing* timing) {
  if (!net) return fail(FFV_ERR_ARG, "null argument");
  if (!net->net.server()) return fail(FFV_ERR_STATE, "serving is off (hbm_budget_bytes = 0)");
  ffv::Timing tm;
  bool done = false;
  ffv_status st = from(net->net.server()->poll(ticket, &tm, &done));
  if (st != FFV_OK) return st;
  if (!done) return FFV_PENDING;
  if (timing) {
    timing->t_submit = tm.t_submit;
    timing->t_admit = tm.t_admit;
    timing->t_launch = tm.t_launch;
    timing->t_done = tm.t_done;
  }
  return FFV_OK;
}

ffv_status ffv_serving_stats(ffv_net* net, int64_t* admitted, int64_t* completed, int64_t* queued,
                             uint64_t* bytes_in_use) {
  if (!net || !admitted || !completed || !queued || !bytes_in_use)
    return fail(FFV_ERR_ARG, "null argument");
  if (!net->net.server()) return fail(FFV_ERR_STATE, "serving is off (hbm_budget_bytes = 0)");
  long a = 0, c = 0, q = 0;
  size_t b = 0;
  ffv_status st = from(net->net.server()->stats(&a, &c, &q, &b));
  *admitted = a;
  *completed = c;
  *queued = q;
  *bytes_in_use = b;
  return st;
}

ffv_status ffv_debug_tap(ffv_net* net, const char* name, float* dst, size_t capacity_floats,
                         int32_t dims[3]) {
  if (!net || !name || !dst || !dims) return fail(FFV_ERR_ARG, "null argument");
  int d[3] = {0, 0, 0};
  ffv_status st = from(net->net.debug_tap(name, dst, capacity_floats, d));
  dims[0] = d[0];
  dims[1] = d[1];
  dims[2] = d[2];
  return st;
}

ffv_status ffv_set_debug(ffv_net* net, int32_t enable) {
  if (!net) return fail(FFV_ERR_ARG, "null net");
  net->net.set_debug(enable != 0);
  return FFV_OK;
}

ffv_status ffv_set_profiling(ffv_net* net, int32_t enable) {
  if (!net) return fail(FFV_ERR_ARG, "null net");
  net->net.set_profiling(enable != 0);
  return FFV_OK;
}

ffv_status ffv_debug_fault(const char* spec) {
  ffv::fault_arm(spec);
  g_last_error.clear();
  return FFV_OK;
}

ffv_status ffv_kernel_stats(ffv_net* net, const char* name, int64_t* launches, double* ms,
                            double* work) {
  if (!net || !name || !launches || !ms || !work) return fail(FFV_ERR_ARG, "null argument");
  long l = 0;
  ffv_status st = from(net->net.kernel_stats(name, &l, ms, work));
  *launches = l;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Multi-view cluster frame.
extern "C" ffv_status ffv_stitch_cluster(const float* real_view, const float* const* left,
                                         const float* const* right, int32_t n_per_side,
                                         int32_t height, int32_t width, float* out, void* stream) {
  using namespace ffv;
  if (!real_view || !left || !right || !out) return fail(FFV_ERR_ARG, "null argument");
  int g = 0;
  for (int k : {1, 2, 4, 8})
    if (k * k == n_per_side) g = k;
  if (g == 0) return fail(FFV_ERR_ARG, "n_per_side must be 1, 4, 16 or 64");
  if (height <= 0 || width <= 0 || height % g != 0 || width % g != 0)
    return fail(FFV_ERR_ARG, "height and width must be positive multiples of sqrt(n_per_side)");
  if (3L * height * width > (1L << 31)) return fail(FFV_ERR_ARG, "image too large");
  StitchArgs a{};
  a.hr = real_view;
  a.n = n_per_side;
  a.g = g;
  a.H = height;
  a.W = width;
  a.out = out;
  for (int i = 0; i < n_per_side; ++i) {
    if (!left[i] || !right[i]) return fail(FFV_ERR_ARG, "null view pointer");
    a.views[i] = left[i];
    a.views[n_per_side + i] = right[i];
    if (g == 4 && ((reinterpret_cast<uintptr_t>(left[i]) | reinterpret_cast<uintptr_t>(right[i])) & 15))
      return fail(FFV_ERR_ARG, "views must be 16-byte aligned");
  }
  const hipError_t err = launch_stitch(a, (hipStream_t)stream);
  if (err != hipSuccess) return fail(FFV_ERR_DEVICE, hipGetErrorString(err));
  g_last_error.clear();
  return FFV_OK;
}

// ---------------------------------------------------------------------------
// Operator-level entry point (kernel unit tests).
namespace ffv {

ffv_status op_fail(int code, const char* msg) { return fail(code, msg); }

ffv_status op_conv_run(const OpConvScratch* scratch, int32_t precision, const float* x, int32_t n,
                       int32_t cin, int32_t h, int32_t w, const float* weight, const float* bias,
                       int32_t cout, int32_t stride, int32_t transposed, int32_t relu, int32_t n_tile,
                       int32_t tile_w, float* y, void* stream) {
  if (!x || !weight || !bias || !y) return fail(FFV_ERR_ARG, "null argument");
  const bool act_out = (precision & FFV_OP_ACT_OUT) != 0;
  precision &= ~FFV_OP_ACT_OUT;
  if (precision != FFV_FP32 && precision != FFV_BF16) return fail(FFV_ERR_ARG, "precision");
  if (n <= 0 || cin <= 0 || h <= 0 || w <= 0 || cout <= 0) return fail(FFV_ERR_ARG, "sizes");
  if (!transposed && stride != 1 && stride != 2) return fail(FFV_ERR_ARG, "stride");
  if (n_tile != 0 && (n_tile < 1 || n_tile > 10) && n_tile != 32 && n_tile != 64 && n_tile != 128 &&
      n_tile != 256)
    return fail(FFV_ERR_ARG, "n_tile must be 0, 1-10, 32, 64, 128 or 256");
  if (tile_w < 0 || tile_w > 256 || (tile_w > 0 && 256 % tile_w != 0))
    return fail(FFV_ERR_ARG, "tile_w must be 0 or divide 256");
  const DType dt = precision == FFV_FP32 ? DType::F32 : DType::BF16;
  hipStream_t s = (hipStream_t)stream;
  Layer L;
  L.transposed = transposed != 0;
  L.cin = cin;
  L.cout = cout;
  L.stride = L.transposed ? 2 : stride;
  const size_t nw = (size_t)cin * cout * (L.transposed ? 16 : 9);
  L.w_host.assign(weight, weight + nw);
  L.b_host.assign(bias, bias + cout);
  plan_layer(L);
  const int ho = L.transposed ? 2 * h : (h - 1) / stride + 1;
  const int wo = L.transposed ? 2 * w : (w - 1) / stride + 1;
  std::vector<uint8_t> packed = pack_layer(L, dt);
  const size_t e = dtype_size(dt);
  // output as the network's layers write it (activation dtype), or float
  const DType out_dt = act_out ? dt : DType::F32;
  // the call's device buffers: NHWC input, packed weights, bias, NHWC output
  // and a zero block for taps outside the image
  const size_t sizes[5] = {(size_t)n * h * w * L.cin_pad * e, packed.size(), (size_t)cout * 4,
                           (size_t)n * ho * wo * cout * dtype_size(out_dt), 256};
  void* buf[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipError_t err = hipSuccess;
  if (scratch) {
    size_t need = 0;
    for (size_t b : sizes) need += (b + 255) / 256 * 256;
    if (need > scratch->cap)
      return fail(FFV_ERR_ARG, "layer needs " + std::to_string(need) + " bytes of scratch; the no-allocation "
                               "entry point holds " + std::to_string(scratch->cap));
    char* p = static_cast<char*>(scratch->base);
    for (int i = 0; i < 5; ++i) {
      buf[i] = p;
      p += (sizes[i] + 255) / 256 * 256;
    }
  } else {
    for (int i = 0; i < 5 && err == hipSuccess; ++i) err = hipMalloc(&buf[i], sizes[i]);
  }
  void *xin = buf[0], *wd = buf[1], *bd = buf[2], *yo = buf[3], *zr = buf[4];
  auto cleanup = [&]() {
    if (scratch) return;
    for (void* b : buf)
      if (b) hipFree(b);
  };
  // (the copies are ordered on s and waited for before returning, so the
  // host vectors they read outlive them)
  if (err == hipSuccess) err = hipMemsetAsync(zr, 0, 256, s);
  if (err == hipSuccess) err = hipMemcpyAsync(wd, packed.data(), packed.size(), hipMemcpyHostToDevice, s);
  if (err == hipSuccess) err = hipMemcpyAsync(bd, bias, (size_t)cout * 4, hipMemcpyHostToDevice, s);
  if (err == hipSuccess) err = launch_pack_nhwc(x, n, cin, h, w, xin, L.cin_pad, dt, s);
  if (err == hipSuccess) {
    ConvArgs a{};
    a.in = xin;
    a.in_img_stride = (long)h * w * L.cin_pad;
    a.in_ld = L.cin_pad;
    a.Hi = h;
    a.Wi = w;
    a.wgt = wd;
    a.bias = (const float*)bd;
    a.out = yo;
    a.out_img_stride = (long)ho * wo * cout;
    a.out_ld = cout;
    a.Ho = L.transposed ? h : ho;
    a.Wo = L.transposed ? w : wo;
    a.Hout = ho;
    a.Wout = wo;
    a.cin_pad = L.cin_pad;
    a.K = L.K;
    a.K_pad = L.K_pad;
    a.cout = cout;
    a.cout_pad = L.cout_pad;
    a.n_rows = L.rows;
    a.n_img = n;
    a.stride = L.transposed ? 1 : stride;
    a.transposed = L.mode;
    a.relu = relu ? 1 : 0;
    a.out_f32 = out_dt == DType::F32 ? 1 : 0;
    a.accumulate = 0;
    a.taps = L.mode == 1 ? 4 : 9;
    a.zero = zr;
    a.tile_w = tile_w > 0 ? tile_w : conv_tile_width(a.Ho, a.Wo);
    ConvTile tile = L.tile;
    if (n_tile == 256) tile = ConvTile::N256;
    if (n_tile == 128) tile = ConvTile::N128;
    if (n_tile == 64) tile = ConvTile::N64;
    if (n_tile == 32) tile = ConvTile::N32;
    if (n_tile == 1) {
      tile = ConvTile::H32;
      a.tile_w = 16;
    }
    if (n_tile == 2) tile = ConvTile::H128;
    if (n_tile == 3) tile = ConvTile::H256;
    if (n_tile == 4 || n_tile == 5) {
      tile = n_tile == 4 ? ConvTile::R32 : ConvTile::R64;
      a.tile_w = 16;
    }
    if (n_tile == 9) tile = ConvTile::Q256;
    if (n_tile == 10) tile = ConvTile::P256;
    if (n_tile >= 6 && n_tile <= 8) {
      tile = n_tile == 6 ? ConvTile::S32 : (n_tile == 7 ? ConvTile::S64 : ConvTile::S128);
      a.tile_w = 16;
    }
    err = launch_conv(dt, tile, a, s);
  }
  for (int i = 0; err == hipSuccess && i < n; ++i)
    err = launch_extract((const char*)yo + (size_t)i * ho * wo * cout * dtype_size(out_dt), out_dt, cout, cout,
                         (long)ho * wo, y + (size_t)i * cout * ho * wo, s);
  // on an error the queued work still reads the buffers: wait before freeing
  const hipError_t sync = hipStreamSynchronize(s);
  if (err == hipSuccess) err = sync;
  cleanup();
  if (err != hipSuccess) return fail(FFV_ERR_DEVICE, hipGetErrorString(err));
  g_last_error.clear();
  return FFV_OK;
}

}  // namespace ffv

extern "C" ffv_status ffv_op_conv(int32_t precision, const float* x, int32_t n, int32_t cin,
                                  int32_t h, int32_t w, const float* weight, const float* bias,
                                  int32_t cout, int32_t stride, int32_t transposed, int32_t relu,
                                  int32_t n_tile, int32_t tile_w, float* y, void* stream) {
  return ffv::op_conv_run(nullptr, precision, x, n, cin, h, w, weight, bias, cout, stride, transposed, relu,
                          n_tile, tile_w, y, stream);
}

extern "C" ffv_status ffv_lap_loss(const float* x, const float* gt, int32_t n, int32_t height, int32_t width,
                                   float* loss, float* grad, void* stream) {
  using namespace ffv;
  if (!x || !gt || !loss) return fail(FFV_ERR_ARG, "null argument");
  if (n <= 0) return fail(FFV_ERR_ARG, "n must be positive");
  if (height < kLapMinSize || width < kLapMinSize)
    return fail(FFV_ERR_ARG, "height and width must be >= " + std::to_string(kLapMinSize));
  if ((long)height * width > (1L << 28)) return fail(FFV_ERR_ARG, "image too large");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = lap_workspace_bytes(n, height, width, grad != nullptr);
  void* ws = nullptr;
  if (fault_hit("alloc") || hipMalloc(&ws, bytes) != hipSuccess) return fail(FFV_ERR_OOM, "workspace");
  hipError_t err = launch_lap_loss(x, gt, n, height, width, loss, grad, ws, bytes, s);
  // wait before freeing: queued kernels read the workspace
  const hipError_t sync = hipStreamSynchronize(s);
  if (err == hipSuccess) err = sync;
  hipFree(ws);
  if (err != hipSuccess) return fail(FFV_ERR_DEVICE, hipGetErrorString(err));
  g_last_error.clear();
  return FFV_OK;
}
