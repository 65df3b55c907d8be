// Network executor for the view-interpolation network (paper section 3.1,
// Eq. 1 and Eq. 2, supplementary layer table).
//
// Per call: every distinct camera image is ingested once (replicate-padded
// to a multiple of 16, NHWC), its quarter/half-size copies and its
// ContextNet features are computed once, and then the (pair, t) views run in
// batched launches: each layer is one launch over all views of a chunk, with
// the views folded into the GEMM's M dimension.
#include "net.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

#include "sha256.h"

namespace ffv {

namespace {

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// float -> bf16 bits, round to nearest even (NaN kept quiet).
inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Expect {
  const char* kind;
  int cin, cout, stride;
};

// The network's own layer definition (section 3.1 and the supplementary
// layer table); the weights file must match it.
std::map<std::string, Expect> expected_layers(int B, bool tp) {
  std::map<std::string, Expect> m;
  const int t = tp ? 1 : 0;
  char buf[64];
  for (int s = 0; s < 3; ++s) {
    snprintf(buf, sizeof buf, "vib%d.conv1", s);
    m[buf] = {"conv", (s == 0 ? 6 : 17) + t, 4 * B, 2};
    snprintf(buf, sizeof buf, "vib%d.conv2", s);
    m[buf] = {"conv", 4 * B, 8 * B, 2};
    for (int i = 3; i <= 8; ++i) {
      snprintf(buf, sizeof buf, "vib%d.conv%d", s, i);
      m[buf] = {"conv", 8 * B, 8 * B, 1};
    }
    snprintf(buf, sizeof buf, "vib%d.convT1", s);
    m[buf] = {"convT", 8 * B, 4 * B, 2};
    snprintf(buf, sizeof buf, "vib%d.convT2", s);
    m[buf] = {"convT", 4 * B, 5, 2};
  }
  const int cw[4] = {B / 2, B, 2 * B, 4 * B};
  int cin = 3;
  for (int k = 0; k < 4; ++k) {
    snprintf(buf, sizeof buf, "ctx.conv%d", 2 * k + 1);
    m[buf] = {"conv", cin, cw[k], 2};
    snprintf(buf, sizeof buf, "ctx.conv%d", 2 * k + 2);
    m[buf] = {"conv", cw[k], cw[k], 1};
    cin = cw[k];
  }
  const int ew[4] = {B, 2 * B, 4 * B, 8 * B};
  const int ei[4] = {17, 2 * B, 4 * B, 8 * B};
  for (int k = 0; k < 4; ++k) {
    snprintf(buf, sizeof buf, "unet.enc%d", 2 * k + 1);
    m[buf] = {"conv", ei[k], ew[k], 2};
    snprintf(buf, sizeof buf, "unet.enc%d", 2 * k + 2);
    m[buf] = {"conv", ew[k], ew[k], 1};
  }
  const int di[4] = {16 * B, 8 * B, 4 * B, 2 * B};
  const int dout[4] = {4 * B, 2 * B, B, B / 2};
  for (int k = 0; k < 4; ++k) {
    snprintf(buf, sizeof buf, "unet.dec%d", k + 1);
    m[buf] = {"convT", di[k], dout[k], 2};
  }
  m["unet.head"] = {"conv", B / 2, 3, 1};
  return m;
}

}  // namespace

Status read_weights_file(const std::string& path, WeightsFile& out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return Status::err(-5, "cannot open weights file: " + path);
  std::vector<char> raw((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (raw.size() < 16 || std::memcmp(raw.data(), "FFVW", 4) != 0)
    return Status::err(-5, "not an FFVW weights file");
  uint32_t version, hlen;
  std::memcpy(&version, raw.data() + 4, 4);
  std::memcpy(&hlen, raw.data() + 8, 4);
  if (version != 1) return Status::err(-5, "unsupported weights version");
  if (16 + (size_t)hlen > raw.size()) return Status::err(-5, "truncated header");
  std::string text(raw.data() + 16, hlen);
  const size_t start = align_up(16 + hlen, 64);
  std::istringstream is(text);
  std::string line, sha;
  long n_floats = -1;
  int n_layers = -1;
  bool ended = false;
  struct Row {
    std::string name, kind;
    int cin, cout, stride;
    long wo, wc, bo, bc;
  };
  std::vector<Row> rows;
  out.base_width = -1;
  int tp = -1;
  while (std::getline(is, line)) {
    std::istringstream ls(line);
    std::string key;
    if (!(ls >> key)) continue;
    if (key == "base_width") ls >> out.base_width;
    else if (key == "t_plane") ls >> tp;
    else if (key == "seed") { long s; ls >> s; }
    else if (key == "n_floats") ls >> n_floats;
    else if (key == "sha256") ls >> sha;
    else if (key == "layers") ls >> n_layers;
    else if (key == "layer") {
      Row r;
      if (!(ls >> r.name >> r.kind >> r.cin >> r.cout >> r.stride >> r.wo >> r.wc >> r.bo >> r.bc))
        return Status::err(-5, "malformed layer line");
      rows.push_back(r);
    } else if (key == "end") { ended = true; break; }
    else return Status::err(-5, "unknown header key: " + key);
  }
  if (!ended || out.base_width <= 0 || tp < 0 || n_floats < 0 || sha.size() != 64 ||
      n_layers != (int)rows.size())
    return Status::err(-5, "incomplete weights header");
  out.t_plane = tp != 0;
  const size_t payload_bytes = (size_t)n_floats * 4;
  if (start + payload_bytes > raw.size()) return Status::err(-5, "truncated payload");
  const uint8_t* pay = reinterpret_cast<const uint8_t*>(raw.data() + start);
  if (sha256_hex(pay, payload_bytes) != sha) return Status::err(-5, "weights checksum mismatch");
  const float* fl = reinterpret_cast<const float*>(pay);

  auto exp = expected_layers(out.base_width, out.t_plane);
  if (exp.size() != rows.size()) return Status::err(-5, "wrong number of layers");
  for (const Row& r : rows) {
    auto it = exp.find(r.name);
    if (it == exp.end()) return Status::err(-5, "unexpected layer " + r.name);
    const Expect& e = it->second;
    if (r.kind != e.kind || r.cin != e.cin || r.cout != e.cout || r.stride != e.stride)
      return Status::err(-5, "layer shape mismatch: " + r.name);
    const long taps = r.kind == "conv" ? 9 : 16;
    if (r.wc != (long)r.cin * r.cout * taps || r.bc != r.cout || r.wo < 0 || r.bo < 0 ||
        r.wo + r.wc > n_floats || r.bo + r.bc > n_floats)
      return Status::err(-5, "layer extent mismatch: " + r.name);
    Layer L;
    L.name = r.name;
    L.transposed = r.kind == "convT";
    L.cin = r.cin;
    L.cout = r.cout;
    L.stride = r.stride;
    L.w_host.assign(fl + r.wo, fl + r.wo + r.wc);
    L.b_host.assign(fl + r.bo, fl + r.bo + r.bc);
    for (float v : L.w_host)
      if (!std::isfinite(v)) return Status::err(-5, "non-finite weight in " + r.name);
    out.layers[r.name] = std::move(L);
  }
  return Status::ok();
}

void plan_layer(Layer& L) {
  L.cin_pad = round_up(L.cin, 8);
  // Transposed convs with few output channels run phase-merged: the four
  // output phases share one 3x3-neighbourhood input tile (N = 4 * cout).
  L.mode = L.transposed ? (L.cout <= 16 ? 2 : 1) : 0;
  L.K = (L.mode == 1 ? 4 : 9) * L.cin_pad;
  L.K_pad = round_up(L.K, 64);  // a multiple of every dtype's K step
  const int n = L.mode == 2 ? 4 * L.cout : L.cout;
  const int bn = n > 128 ? 256 : (n > 64 ? 128 : (n > 32 ? 64 : 32));
  L.tile = bn == 256 ? ConvTile::N256
                     : (bn == 128 ? ConvTile::N128 : (bn == 64 ? ConvTile::N64 : ConvTile::N32));
  L.cout_pad = round_up(n, bn);
}

std::vector<uint8_t> pack_layer(const Layer& L, DType dt) {
  const int phases = L.mode == 1 ? 4 : 1;
  const size_t n = (size_t)phases * L.cout_pad * L.K_pad;
  std::vector<float> p(n, 0.f);
  if (L.mode == 0) {
    // k = (dy*3 + dx) * cin_pad + c  <-  w[o][c][dy][dx]
    for (int o = 0; o < L.cout; ++o) {
      float* row = &p[(size_t)o * L.K_pad];
      for (int c = 0; c < L.cin; ++c)
        for (int tap = 0; tap < 9; ++tap)
          row[tap * L.cin_pad + c] = L.w_host[((size_t)o * L.cin + c) * 9 + tap];
    }
  } else if (L.mode == 1) {
    // phase (py, px), tap (ty, tx) reads input (a + py - ty, b + px - tx) with
    // kernel index (1 - py + 2ty, 1 - px + 2tx);
    // k = (ty*2 + tx) * cin_pad + c  <-  w[c][o][ky][kx]
    for (int ph = 0; ph < 4; ++ph) {
      const int py = ph >> 1, px = ph & 1;
      for (int o = 0; o < L.cout; ++o) {
        float* row = &p[((size_t)ph * L.cout_pad + o) * L.K_pad];
        for (int c = 0; c < L.cin; ++c)
          for (int ty = 0; ty < 2; ++ty)
            for (int tx = 0; tx < 2; ++tx) {
              const int ky = 1 - py + 2 * ty, kx = 1 - px + 2 * tx;
              row[(ty * 2 + tx) * L.cin_pad + c] =
                  L.w_host[(((size_t)c * L.cout + o) * 4 + ky) * 4 + kx];
            }
      }
    }
  } else {
    // phase-merged: row n = ph * cout + o, k = ((dy+1)*3 + (dx+1)) * cin_pad + c
    // over the input's 3x3 neighbourhood; phase (py, px) uses the taps with
    // ty = py - dy and tx = px - dx in {0, 1}, kernel index (1 - py + 2ty, 1 - px + 2tx).
    for (int ph = 0; ph < 4; ++ph) {
      const int py = ph >> 1, px = ph & 1;
      for (int o = 0; o < L.cout; ++o) {
        float* row = &p[((size_t)ph * L.cout + o) * L.K_pad];
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int ty = py - dy, tx = px - dx;
            if (ty < 0 || ty > 1 || tx < 0 || tx > 1) continue;
            const int ky = 1 - py + 2 * ty, kx = 1 - px + 2 * tx;
            const int tap = (dy + 1) * 3 + (dx + 1);
            for (int c = 0; c < L.cin; ++c)
              row[tap * L.cin_pad + c] = L.w_host[(((size_t)c * L.cout + o) * 4 + ky) * 4 + kx];
          }
      }
    }
  }
  std::vector<uint8_t> bytes;
  if (dt == DType::F32) {
    bytes.resize(n * 4);
    std::memcpy(bytes.data(), p.data(), n * 4);
  } else {
    bytes.resize(n * 2);
    uint16_t* q = reinterpret_cast<uint16_t*>(bytes.data());
    for (size_t i = 0; i < n; ++i) q[i] = f2bf(p[i]);
  }
  return bytes;
}

// ----------------------------------------------------------------- Net

Net::~Net() {
  if (device_ >= 0) hipSetDevice(device_);
  if (stream_) hipStreamSynchronize(stream_);
  for (auto& kv : layers_) {
    if (kv.second.w_dev) hipFree(kv.second.w_dev);
    if (kv.second.b_dev) hipFree(kv.second.b_dev);
  }
  if (ws_) hipFree(ws_);
  if (src_ptrs_) hipFree(src_ptrs_);
  for (auto& e : pending_) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  for (auto e : evt_pool_) hipEventDestroy(e);
  if (own_stream_ && stream_) hipStreamDestroy(stream_);
}

Status Net::check(hipError_t e, const char* what) {
  if (e == hipSuccess) return Status::ok();
  const int code = (e == hipErrorOutOfMemory) ? -2 : -4;
  return Status::err(code, std::string(what) + ": " + hipGetErrorString(e));
}

Status Net::init(const std::string& path, int precision, int device, hipStream_t stream,
                 size_t workspace_cap) {
  if (precision != 0 && precision != 1)
    return Status::err(-1, "precision not supported (FP32 = 0 and BF16 = 1 are built)");
  dt_ = precision == 0 ? DType::F32 : DType::BF16;
  device_ = device;
  ws_cap_ = workspace_cap ? workspace_cap : (size_t)16 << 30;
  WeightsFile wf;
  Status st = read_weights_file(path, wf);
  if (!st.good()) return st;
  base_width_ = wf.base_width;
  t_plane_ = wf.t_plane;
  if (base_width_ % 16 != 0 || base_width_ > 128)
    return Status::err(-5, "base width must be a multiple of 16, at most 128, for the GPU layouts");
  int ndev = 0;
  st = check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (!st.good()) return st;
  if (device < 0 || device >= ndev) return Status::err(-1, "device ordinal out of range");
  st = check(hipSetDevice(device), "hipSetDevice");
  if (!st.good()) return st;
  if (stream) {
    stream_ = stream;
  } else {
    st = check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "hipStreamCreate");
    if (!st.good()) return st;
    own_stream_ = true;
  }
  layers_ = std::move(wf.layers);
  for (auto& kv : layers_) {
    Layer& L = kv.second;
    plan_layer(L);
    if (L.name == "unet.head") continue;  // evaluated by the head kernel in fp32
    std::vector<uint8_t> packed = pack_layer(L, dt_);
    st = check(hipMalloc(&L.w_dev, packed.size()), "hipMalloc weights");
    if (!st.good()) return st;
    st = check(hipMemcpy(L.w_dev, packed.data(), packed.size(), hipMemcpyHostToDevice), "copy weights");
    if (!st.good()) return st;
  }
  for (auto& kv : layers_) {
    Layer& L = kv.second;
    const std::vector<float>& src = L.b_host;
    st = check(hipMalloc((void**)&L.b_dev, src.size() * 4), "hipMalloc bias");
    if (!st.good()) return st;
    st = check(hipMemcpy(L.b_dev, src.data(), src.size() * 4, hipMemcpyHostToDevice), "copy bias");
    if (!st.good()) return st;
  }
  {
    // head weights stay fp32 in file layout [3][16][3][3]
    Layer& H = layers_.at("unet.head");
    st = check(hipMalloc(&H.w_dev, H.w_host.size() * 4), "hipMalloc head");
    if (!st.good()) return st;
    st = check(hipMemcpy(H.w_dev, H.w_host.data(), H.w_host.size() * 4, hipMemcpyHostToDevice),
               "copy head");
    if (!st.good()) return st;
  }
  return Status::ok();
}

Status Net::make_plan(const Geo& g, int n_cam, int n_view, Plan& p) const {
  const size_t e = dtype_size(dt_);
  const long P = g.P;
  const int B = base_width_;
  const size_t A = 256;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, A);
    return o;
  };
  p.g = g;
  p.n_cam = n_cam;
  p.n_view = n_view;
  const size_t C = n_cam, V = n_view;
  p.X4 = take(C * P * 4 * 4);
  p.Xa = take(C * P * 8 * e);
  p.L0 = take(C * (P / 16) * 4 * 4);
  p.L1 = take(C * (P / 4) * 4 * 4);
  const int cw[4] = {B / 2, B, 2 * B, 4 * B};
  for (int k = 0; k < 4; ++k) p.ctx[k] = take(C * (P >> (2 * (k + 1))) * cw[k] * e);
  p.ctmp = take(C * (P / 4) * (B / 2) * e);
  p.FM[0] = take(V * (P / 16) * 8 * 4);
  p.FM[1] = take(V * (P / 4) * 8 * 4);
  p.FM[2] = take(V * P * 8 * 4);
  p.I2 = take(V * P * 4 * 4);
  for (int k = 0; k < 4; ++k) p.Fp[k] = take(V * (P >> (2 * (k + 1))) * 4 * 4);
  p.views = take(V * sizeof(ViewDesc));
  const size_t phase0 = off;
  // VIBlock region
  p.xin = take(V * P * 24 * e);
  p.a1 = take(V * (P / 4) * 4 * B * e);
  p.bA = take(V * (P / 16) * 8 * B * e);
  p.bB = take(V * (P / 16) * 8 * B * e);
  const size_t end_vib = off;
  off = phase0;
  // U-Net region (aliases the VIBlock region)
  p.x0u = take(V * P * 24 * e);
  const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
  for (int k = 0; k < 4; ++k) p.lvl[k] = take(V * (P >> (2 * (k + 1))) * lv_ld[k] * e);
  p.etmp = take(V * (P / 4) * B * e);
  p.u4 = take(V * P * (B / 2) * e);
  p.total = std::max(off, end_vib);
  return Status::ok();
}

Status Net::ensure_workspace(size_t bytes) {
  if (bytes <= ws_bytes_) return Status::ok();
  if (ws_) {
    hipStreamSynchronize(stream_);
    hipFree(ws_);
    ws_ = nullptr;
    ws_bytes_ = 0;
  }
  Status st = check(hipMalloc(&ws_, bytes), "hipMalloc workspace");
  if (!st.good()) return st;
  ws_bytes_ = bytes;
  return Status::ok();
}

void Net::set_profiling(bool on) {
  profiling_ = on;
  stats_.clear();
}

void Net::prof_begin() {
  if (!profiling_) return;
  hipEvent_t e;
  if (!evt_pool_.empty()) {
    e = evt_pool_.back();
    evt_pool_.pop_back();
  } else {
    hipEventCreate(&e);
  }
  hipEventRecord(e, stream_);
  cur_start_ = e;
}

void Net::prof_end(const char* cls, double work) {
  if (!profiling_ || !cur_start_) return;
  hipEvent_t e;
  if (!evt_pool_.empty()) {
    e = evt_pool_.back();
    evt_pool_.pop_back();
  } else {
    hipEventCreate(&e);
  }
  hipEventRecord(e, stream_);
  pending_.push_back({cur_start_, e, cls, work});
  cur_start_ = nullptr;
}

Status Net::kernel_stats(const std::string& name, long* launches, double* ms, double* work) {
  auto it = stats_.find(name);
  if (it == stats_.end()) {
    *launches = 0;
    *ms = 0;
    *work = 0;
    return Status::ok();
  }
  *launches = it->second.launches;
  *ms = it->second.ms;
  *work = it->second.work;
  return Status::ok();
}

Status Net::conv(const Layer& L, const void* in, int in_ld, long in_img_stride, int Hi, int Wi,
                 int n_img, void* out, int out_ld, long out_img_stride, bool out_f32,
                 bool accumulate, bool relu) {
  ConvArgs a{};
  a.in = in;
  a.in_img_stride = in_img_stride;
  a.in_ld = in_ld;
  a.Hi = Hi;
  a.Wi = Wi;
  a.wgt = L.w_dev;
  a.bias = L.b_dev;
  a.out = out;
  a.out_img_stride = out_img_stride;
  a.out_ld = out_ld;
  if (L.transposed) {
    a.Ho = Hi;
    a.Wo = Wi;
    a.Hout = 2 * Hi;
    a.Wout = 2 * Wi;
  } else {
    a.Ho = (Hi - 1) / L.stride + 1;
    a.Wo = (Wi - 1) / L.stride + 1;
    a.Hout = a.Ho;
    a.Wout = a.Wo;
  }
  a.cin_pad = L.cin_pad;
  a.K = L.K;
  a.K_pad = L.K_pad;
  a.cout = L.cout;
  a.cout_pad = L.cout_pad;
  a.n_img = n_img;
  a.stride = L.transposed ? 1 : L.stride;
  a.transposed = L.mode;
  a.relu = relu ? 1 : 0;
  a.out_f32 = out_f32 ? 1 : 0;
  a.accumulate = accumulate ? 1 : 0;
  if (in_ld < L.cin_pad || in_ld % 8 != 0) return Status::err(-4, "conv input stride");
  const double flops = 2.0 * n_img * (double)a.Hout * a.Wout * L.cout * L.cin *
                       (L.transposed ? 4.0 : 9.0);
  const char* cls = L.transposed ? "convT"
                                 : ((L.cin == 8 * base_width_ && L.cout == 8 * base_width_ &&
                                     L.stride == 1)
                                        ? "conv256"
                                        : "conv");
  prof_begin();
  Status st = check(launch_conv(dt_, L.tile, a, stream_), L.name.c_str());
  prof_end(cls, flops);
  return st;
}

#define FFV_TRY(expr)              \
  do {                             \
    Status _s = (expr);            \
    if (!_s.good()) return _s;     \
  } while (0)

Status Net::interpolate(const float* const* left, const float* const* right, int n_pairs, int H,
                        int W, const float* t, int n_t, float* out) {
  FFV_TRY(check(hipSetDevice(device_), "hipSetDevice"));
  Geo g;
  g.H = H;
  g.W = W;
  g.Hp = round_up(H, 16);
  g.Wp = round_up(W, 16);
  g.P = (long)g.Hp * g.Wp;

  // distinct cameras
  std::vector<const float*> cams;
  std::vector<int> li(n_pairs), ri(n_pairs);
  auto slot = [&](const float* p) {
    for (size_t i = 0; i < cams.size(); ++i)
      if (cams[i] == p) return (int)i;
    cams.push_back(p);
    return (int)cams.size() - 1;
  };
  for (int i = 0; i < n_pairs; ++i) {
    li[i] = slot(left[i]);
    ri[i] = slot(right[i]);
  }
  const int n_cam = (int)cams.size();
  const int n_view_total = n_pairs * n_t;

  // chunk size: as many views as fit the workspace cap
  Plan one;
  FFV_TRY(make_plan(g, n_cam, 1, one));
  Plan two;
  FFV_TRY(make_plan(g, n_cam, 2, two));
  const size_t per_view = two.total - one.total;
  const size_t fixed = one.total - per_view;
  int chunk = n_view_total;
  if (!debug_ && fixed + per_view * (size_t)chunk > ws_cap_) {
    chunk = (int)std::max<size_t>(1, (ws_cap_ > fixed ? (ws_cap_ - fixed) / per_view : 1));
  }
  chunk = std::min(chunk, n_view_total);
  Plan p;
  FFV_TRY(make_plan(g, n_cam, chunk, p));
  FFV_TRY(ensure_workspace(p.total));

  // camera pointer table
  if (src_ptrs_cap_ < (size_t)n_cam) {
    if (src_ptrs_) hipFree(src_ptrs_);
    src_ptrs_ = nullptr;
    FFV_TRY(check(hipMalloc(&src_ptrs_, sizeof(void*) * n_cam), "hipMalloc ptrs"));
    src_ptrs_cap_ = n_cam;
  }
  FFV_TRY(check(hipMemcpyAsync(src_ptrs_, cams.data(), sizeof(void*) * n_cam, hipMemcpyHostToDevice,
                               stream_),
                "copy ptrs"));

  const long P = g.P;
  const int B = base_width_;
  const size_t e = dtype_size(dt_);
  float* X4 = (float*)ws(p.X4);
  // 1. ingest + pad, image pyramid
  prof_begin();
  FFV_TRY(check(launch_ingest((const float* const*)src_ptrs_, n_cam, H, W, g.Hp, g.Wp, X4, ws(p.Xa),
                              dt_, stream_),
                "ingest"));
  prof_end("pixel", (double)n_cam * (H * (double)W * 12 + P * (16.0 + 8 * e)));
  prof_begin();
  FFV_TRY(check(launch_resample4(X4, n_cam, g.Hp, g.Wp, (float*)ws(p.L0), g.Hp / 4, g.Wp / 4, stream_),
                "resample L0"));
  FFV_TRY(check(launch_resample4(X4, n_cam, g.Hp, g.Wp, (float*)ws(p.L1), g.Hp / 2, g.Wp / 2, stream_),
                "resample L1"));
  prof_end("pixel", (double)n_cam * (2 * P * 16.0 + (P / 16 + P / 4) * 16.0));

  // 2. ContextNet over all cameras
  {
    const int cw[4] = {B / 2, B, 2 * B, 4 * B};
    const void* src = ws(p.Xa);
    int src_ld = 8, h = g.Hp, w = g.Wp;
    for (int k = 0; k < 4; ++k) {
      const int ho = h / 2, wo = w / 2;
      char n1[32], n2[32];
      snprintf(n1, sizeof n1, "ctx.conv%d", 2 * k + 1);
      snprintf(n2, sizeof n2, "ctx.conv%d", 2 * k + 2);
      FFV_TRY(conv(layer(n1), src, src_ld, (long)h * w * src_ld, h, w, n_cam, ws(p.ctmp), cw[k],
                   (long)ho * wo * cw[k], false, false, true));
      FFV_TRY(conv(layer(n2), ws(p.ctmp), cw[k], (long)ho * wo * cw[k], ho, wo, n_cam, ws(p.ctx[k]),
                   cw[k], (long)ho * wo * cw[k], false, false, true));
      src = ws(p.ctx[k]);
      src_ld = cw[k];
      h = ho;
      w = wo;
    }
  }

  // 3. views, in chunks
  std::vector<ViewDesc> vd(n_view_total);
  for (int i = 0; i < n_pairs; ++i)
    for (int j = 0; j < n_t; ++j) vd[(size_t)i * n_t + j] = {li[i], ri[i], t[j], 0};
  std::vector<float*> outs(n_view_total);
  for (int v = 0; v < n_view_total; ++v) outs[v] = out + (size_t)v * 3 * H * W;
  for (int v0 = 0; v0 < n_view_total; v0 += chunk) {
    const int nv = std::min(chunk, n_view_total - v0);
    FFV_TRY(run_chunk(p, vd.data() + v0, nv, outs.data() + v0));
  }
  (void)e;
  FFV_TRY(check(hipStreamSynchronize(stream_), "hipStreamSynchronize"));
  last_plan_ = p;
  have_taps_ = true;
  if (profiling_) {
    for (auto& pe : pending_) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, pe.a, pe.b);
      KernelStat& ks = stats_[pe.cls];
      ks.launches += 1;
      ks.ms += ms;
      ks.work += pe.work;
      evt_pool_.push_back(pe.a);
      evt_pool_.push_back(pe.b);
    }
    pending_.clear();
  }
  return Status::ok();
}

Status Net::run_chunk(const Plan& p, const ViewDesc* views_host, int nv, float* const* outs) {
  const Geo& g = p.g;
  const long P = g.P;
  const int B = base_width_;
  const size_t e = dtype_size(dt_);
  ViewDesc* views = (ViewDesc*)ws(p.views);
  FFV_TRY(check(hipMemcpyAsync(views, views_host, sizeof(ViewDesc) * nv, hipMemcpyHostToDevice,
                               stream_),
                "copy views"));
  const int tp = t_plane_ ? 1 : 0;

  // stage 0 input
  const int h0 = g.Hp / 4, w0 = g.Wp / 4;
  prof_begin();
  FFV_TRY(check(launch_assemble0(views, nv, (const float*)ws(p.L0), (P / 16) * 4, h0, w0, ws(p.xin), 8,
                                 dt_, tp, stream_),
                "assemble0"));
  prof_end("pixel", (double)nv * (P / 16) * (32.0 + 8 * e));

  for (int s = 0; s < 3; ++s) {
    const int h = g.Hp * (1 << s) / 4, w = g.Wp * (1 << s) / 4;
    const long Ps = (long)h * w;
    const int in_ld = s == 0 ? 8 : 24;
    char nm[32];
    auto L = [&](const char* suffix) -> const Layer& {
      snprintf(nm, sizeof nm, "vib%d.%s", s, suffix);
      return layer(nm);
    };
    if (s > 0) {
      const int hp = h / 2, wp = w / 2;
      const float* Limg = s == 1 ? (const float*)ws(p.L1) : (const float*)ws(p.X4);
      const long cam_stride = s == 1 ? (P / 4) * 4 : P * 4;
      prof_begin();
      FFV_TRY(check(launch_transition(views, nv, (const float*)ws(p.FM[s - 1]), hp, wp, Limg,
                                      cam_stride, h, w, ws(p.xin), 24, (float*)ws(p.FM[s]), dt_, tp,
                                      stream_),
                    "transition"));
      prof_end("pixel", (double)nv * Ps * (20.0 / 4 + 16 * 4 + 24 * e + 32));
    }
    // VIBlock_s
    const int h1 = h / 2, w1 = w / 2, h2 = h / 4, w2 = w / 4;
    const int C1 = 4 * B, C2 = 8 * B;
    FFV_TRY(conv(L("conv1"), ws(p.xin), in_ld, Ps * in_ld, h, w, nv, ws(p.a1), C1, (long)h1 * w1 * C1,
                 false, false, true));
    FFV_TRY(conv(L("conv2"), ws(p.a1), C1, (long)h1 * w1 * C1, h1, w1, nv, ws(p.bA), C2,
                 (long)h2 * w2 * C2, false, false, true));
    void* cur = ws(p.bA);
    void* nxt = ws(p.bB);
    for (int i = 3; i <= 8; ++i) {
      char suf[16];
      snprintf(suf, sizeof suf, "conv%d", i);
      FFV_TRY(conv(L(suf), cur, C2, (long)h2 * w2 * C2, h2, w2, nv, nxt, C2, (long)h2 * w2 * C2, false,
                   false, true));
      std::swap(cur, nxt);
    }
    FFV_TRY(conv(L("convT1"), cur, C2, (long)h2 * w2 * C2, h2, w2, nv, ws(p.a1), C1, (long)h1 * w1 * C1,
                 false, false, true));
    FFV_TRY(conv(L("convT2"), ws(p.a1), C1, (long)h1 * w1 * C1, h1, w1, nv, ws(p.FM[s]), 8, Ps * 8, true,
                 s > 0, false));
  }

  // final warp + blend, U-Net input
  prof_begin();
  FFV_TRY(check(launch_final(views, nv, (const float*)ws(p.FM[2]), (const float*)ws(p.X4), P * 4,
                             g.Hp, g.Wp, (float*)ws(p.I2), ws(p.x0u), 24, dt_, stream_),
                "final"));
  prof_end("pixel", (double)nv * P * (20.0 + 16 * 4 + 16 + 24 * e));

  // flow pyramid and context warps
  {
    const float* src = (const float*)ws(p.FM[2]);
    int ld = 8, h = g.Hp, w = g.Wp;
    const int cw[4] = {B / 2, B, 2 * B, 4 * B};
    const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
    const int lv_off[4] = {2 * B, 4 * B, 8 * B, 8 * B};
    for (int k = 0; k < 4; ++k) {
      const int ho = h / 2, wo = w / 2;
      const long Pk = (long)ho * wo;
      prof_begin();
      FFV_TRY(check(launch_flow_down(src, ld, nv, h, w, (float*)ws(p.Fp[k]), stream_), "flow_down"));
      FFV_TRY(check(launch_ctx_warp(views, nv, ws(p.ctx[k]), Pk * cw[k], cw[k], (const float*)ws(p.Fp[k]),
                                    ho, wo, (char*)ws(p.lvl[k]) + lv_off[k] * e, lv_ld[k],
                                    Pk * lv_ld[k], dt_, stream_),
                    "ctx_warp"));
      prof_end("pixel", (double)nv * ((double)h * w * 16 + Pk * 16 + 2 * Pk * 16 +
                                      2.0 * Pk * cw[k] * e * 2));
      src = (const float*)ws(p.Fp[k]);
      ld = 4;
      h = ho;
      w = wo;
    }
  }

  // context-aware U-Net
  {
    const int ew[4] = {B, 2 * B, 4 * B, 8 * B};
    const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
    // encoder: level k reads [d_k, wc_k] (channels [ew[k-1], ...) of lvl[k-1]) or x0u
    const void* src = ws(p.x0u);
    int src_ld = 24, h = g.Hp, w = g.Wp;
    for (int k = 0; k < 4; ++k) {
      const int ho = h / 2, wo = w / 2;
      char n1[32], n2[32];
      snprintf(n1, sizeof n1, "unet.enc%d", 2 * k + 1);
      snprintf(n2, sizeof n2, "unet.enc%d", 2 * k + 2);
      FFV_TRY(conv(layer(n1), src, src_ld, (long)h * w * src_ld, h, w, nv, ws(p.etmp), ew[k],
                   (long)ho * wo * ew[k], false, false, true));
      // d_{k+1} goes after the decoder slot in lvl[k] (offset ew[k] for k < 3, 0 for the deepest)
      const int d_off = k < 3 ? ew[k] : 0;
      char* dst = (char*)ws(p.lvl[k]) + (size_t)d_off * e;
      FFV_TRY(conv(layer(n2), ws(p.etmp), ew[k], (long)ho * wo * ew[k], ho, wo, nv, dst, lv_ld[k],
                   (long)ho * wo * lv_ld[k], false, false, true));
      src = dst;
      src_ld = lv_ld[k];
      h = ho;
      w = wo;
    }
    // decoder
    const int dout[4] = {4 * B, 2 * B, B, B / 2};
    for (int k = 0; k < 4; ++k) {
      const int lvl_in = 3 - k;  // lvl[3] .. lvl[0]
      const int hi = g.Hp >> (lvl_in + 1), wi = g.Wp >> (lvl_in + 1);
      const void* in = ws(p.lvl[lvl_in]);
      char nm[32];
      snprintf(nm, sizeof nm, "unet.dec%d", k + 1);
      void* dst;
      int dst_ld;
      long dst_stride;
      if (k < 3) {
        dst = ws(p.lvl[lvl_in - 1]);
        dst_ld = lv_ld[lvl_in - 1];
      } else {
        dst = ws(p.u4);
        dst_ld = B / 2;
      }
      dst_stride = (long)(2 * hi) * (2 * wi) * dst_ld;
      (void)dout;
      FFV_TRY(conv(layer(nm), in, lv_ld[lvl_in], (long)hi * wi * lv_ld[lvl_in], hi, wi, nv, dst, dst_ld,
                   dst_stride, false, false, true));
    }
  }

  // output head
  {
    const Layer& Hd = layer("unet.head");
    // outputs of a chunk are contiguous when the chunk's views are
    float* o = outs[0];
    prof_begin();
    FFV_TRY(check(launch_head(ws(p.u4), B / 2, B / 2, (const float*)Hd.w_dev, Hd.b_dev, (const float*)ws(p.I2),
                              nv, g.Hp, g.Wp, g.H, g.W, o, dt_, stream_),
                  "head"));
    prof_end("head", (double)nv * ((double)P * (B / 2) * e + (double)P * 16 + 12.0 * g.H * g.W));
  }
  return Status::ok();
}

Status Net::debug_tap(const std::string& name, float* dst, size_t cap, int dims[3]) {
  if (!have_taps_) return Status::err(-7, "no forward pass recorded");
  const Plan& p = last_plan_;
  const Geo& g = p.g;
  const void* src;
  int C, ld, h, w;
  DType dt = DType::F32;
  if (name == "F0" || name == "F1" || name == "F2") {
    const int s = name[1] - '0';
    h = g.Hp * (1 << s) / 4;
    w = g.Wp * (1 << s) / 4;
    src = ws(p.FM[s]);
    C = 5;
    ld = 8;
  } else if (name == "I2") {
    h = g.Hp;
    w = g.Wp;
    src = ws(p.I2);
    C = 3;
    ld = 4;
  } else {
    return Status::err(-1, "unknown tap " + name);
  }
  const size_t need = (size_t)C * h * w;
  if (cap < need) return Status::err(-1, "tap buffer too small");
  dims[0] = C;
  dims[1] = h;
  dims[2] = w;
  FFV_TRY(check(launch_extract(src, dt, ld, C, (long)h * w, dst, stream_), "extract"));
  return check(hipStreamSynchronize(stream_), "sync");
}

}  // namespace ffv
