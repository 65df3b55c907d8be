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
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "fault.h"
#include "serve.h"
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
  L.rows = n;
  // rows padded to the widest N tile, so any tile width can run the layer
  L.cout_pad = round_up(n, 256);
}

// Weights (file layout w_file) rearranged as the conv kernel reads them, in
// float: [phase][cout_pad][k_pad] with the kernel's K order for K step bk.
static std::vector<float> pack_layer_f(const Layer& L, int bk, int k_pad,
                                       const std::vector<float>& w_file) {
  const int phases = L.mode == 1 ? 4 : 1;
  const int taps = L.mode == 1 ? 4 : 9;
  const size_t n = (size_t)phases * L.cout_pad * k_pad;
  // K position of (tap, channel): channel-slice major when the channel count
  // is a multiple of the kernel's K step (as the kernel walks K), else tap major.
  const bool slice_major = L.cin_pad % bk == 0;
  auto kpos = [&](int tap, int c) {
    if (!slice_major) return tap * L.cin_pad + c;
    return ((c / bk) * taps + tap) * bk + (c % bk);
  };
  std::vector<float> p(n, 0.f);
  if (L.mode == 0) {
    // tap = dy*3 + dx  <-  w[o][c][dy][dx]
    for (int o = 0; o < L.cout; ++o) {
      float* row = &p[(size_t)o * k_pad];
      for (int c = 0; c < L.cin; ++c)
        for (int tap = 0; tap < 9; ++tap) row[kpos(tap, c)] = w_file[((size_t)o * L.cin + c) * 9 + tap];
    }
  } else if (L.mode == 1) {
    // phase (py, px), tap (ty, tx) reads input (a + py - ty, b + px - tx) with
    // kernel index (1 - py + 2ty, 1 - px + 2tx); tap = ty*2 + tx  <-  w[c][o][ky][kx]
    for (int ph = 0; ph < 4; ++ph) {
      const int py = ph >> 1, px = ph & 1;
      for (int o = 0; o < L.cout; ++o) {
        float* row = &p[((size_t)ph * L.cout_pad + o) * k_pad];
        for (int c = 0; c < L.cin; ++c)
          for (int ty = 0; ty < 2; ++ty)
            for (int tx = 0; tx < 2; ++tx) {
              const int ky = 1 - py + 2 * ty, kx = 1 - px + 2 * tx;
              row[kpos(ty * 2 + tx, c)] = w_file[(((size_t)c * L.cout + o) * 4 + ky) * 4 + kx];
            }
      }
    }
  } else {
    // phase-merged: row n = ph * cout + o, tap = (dy+1)*3 + (dx+1) over the
    // input's 3x3 neighbourhood; phase (py, px) uses the taps with
    // ty = py - dy and tx = px - dx in {0, 1}, kernel index (1 - py + 2ty, 1 - px + 2tx).
    for (int ph = 0; ph < 4; ++ph) {
      const int py = ph >> 1, px = ph & 1;
      for (int o = 0; o < L.cout; ++o) {
        float* row = &p[((size_t)ph * L.cout + o) * k_pad];
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int ty = py - dy, tx = px - dx;
            if (ty < 0 || ty > 1 || tx < 0 || tx > 1) continue;
            const int ky = 1 - py + 2 * ty, kx = 1 - px + 2 * tx;
            const int tap = (dy + 1) * 3 + (dx + 1);
            for (int c = 0; c < L.cin; ++c)
              row[kpos(tap, c)] = w_file[(((size_t)c * L.cout + o) * 4 + ky) * 4 + kx];
          }
      }
    }
  }
  return p;
}

// float -> fp8 e4m3 (OCP: bias 7, max 448, no infinities) byte, saturating,
// round to nearest even.
static uint8_t f2f8(float v) {
  uint8_t sign = std::signbit(v) ? 0x80 : 0;
  float a = std::fabs(v);
  if (!(a == a)) return 0x7f;  // NaN
  if (a >= 448.f) return sign | 0x7e;
  if (a < std::ldexp(1.f, -10)) return sign;  // below half the smallest subnormal
  int e = (int)std::floor(std::log2(a));
  if (e < -6) {  // subnormal: multiples of 2^-9
    const float q = std::nearbyint(a * 512.f);
    if (q >= 8.f) return sign | 0x08;
    return sign | (uint8_t)q;
  }
  float m = a / std::ldexp(1.f, e) - 1.f;  // [0, 1)
  float q = std::nearbyint(m * 8.f);
  if (q >= 8.f) {
    q = 0.f;
    e += 1;
  }
  if (e > 8 || (e == 8 && q > 6.f)) return sign | 0x7e;
  return sign | (uint8_t)((e + 7) << 3) | (uint8_t)q;
}

std::vector<uint8_t> pack_layer(const Layer& L, DType dt) {
  const size_t n = (size_t)(L.mode == 1 ? 4 : 1) * L.cout_pad * L.K_pad;
  std::vector<float> p = pack_layer_f(L, conv_k_step(dt), L.K_pad, L.w_host);
  std::vector<uint8_t> bytes;
  if (dt == DType::FP8) {
    bytes.resize(n);
    for (size_t i = 0; i < n; ++i) bytes[i] = f2f8(p[i]);
  } else if (dt == DType::F32) {
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

Geo Geo::of(int H, int W) {
  Geo g;
  g.H = H;
  g.W = W;
  g.Hp = round_up(H, 16);
  g.Wp = round_up(W, 16);
  g.P = (long)g.Hp * g.Wp;
  return g;
}

Net::Net() = default;

Net::~Net() {
  sched_.reset();
  exec_.reset();
  if (device_ >= 0) hipSetDevice(device_);
  if (stream_) hipStreamSynchronize(stream_);
  drop_graphs();
  for (auto& kv : layers_) {
    Layer& L = kv.second;
    for (void* p : {(void*)L.w_dev, (void*)L.b_dev, L.w8_dev, (void*)L.w8_scale, (void*)L.out_scale,
                    (void*)L.amax})
      if (p) hipFree(p);
  }
  if (ws_) hipFree(ws_);
  if (zero_) hipFree(zero_);
  for (auto& e : pending_) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  for (auto e : evt_pool_) hipEventDestroy(e);
  if (own_stream_ && stream_) hipStreamDestroy(stream_);
}

Status Net::dev_alloc(void** p, size_t bytes, const char* what) const {
  *p = nullptr;
  if (fault_hit("alloc"))
    return Status::err(kErrOom, std::string("hipMalloc ") + what + ": injected fault (FFV_FAULT)");
  return check(hipMalloc(p, bytes), what);
}

Status Net::check(hipError_t e, const char* what) const {
  if (e == hipSuccess) return Status::ok();
  const int code = (e == hipErrorOutOfMemory) ? -2 : -4;
  return Status::err(code, std::string(what) + ": " + hipGetErrorString(e));
}

#define FFV_TRY(expr)              \
  do {                             \
    Status _s = (expr);            \
    if (!_s.good()) return _s;     \
  } while (0)

Status Net::init(const std::string& path, int precision, int device, hipStream_t stream,
                 size_t workspace_cap) {
  if (precision < 0 || precision > 2) return Status::err(-1, "unknown precision");
  dt_ = precision == 0 ? DType::F32 : DType::BF16;
  fp8_ = precision == 2;
  device_ = device;
  ws_cap_ = workspace_cap ? workspace_cap : (size_t)16 << 30;
  WeightsFile wf;
  FFV_TRY(read_weights_file(path, wf));
  base_width_ = wf.base_width;
  t_plane_ = wf.t_plane;
  if (base_width_ % 16 != 0 || base_width_ > 128)
    return Status::err(-5, "base width must be a multiple of 16, at most 128, for the GPU layouts");
  int ndev = 0;
  FFV_TRY(check(hipGetDeviceCount(&ndev), "hipGetDeviceCount"));
  if (device < 0 || device >= ndev) return Status::err(-1, "device ordinal out of range");
  FFV_TRY(check(hipSetDevice(device), "hipSetDevice"));
  if (stream) {
    stream_ = stream;
  } else {
    FFV_TRY(check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "hipStreamCreate"));
    own_stream_ = true;
  }
  FFV_TRY(dev_alloc(&zero_, 256, "zero"));
  FFV_TRY(check(hipMemset(zero_, 0, 256), "hipMemset zero"));
  layers_ = std::move(wf.layers);
  for (auto& kv : layers_) {
    Layer& L = kv.second;
    plan_layer(L);
    if (L.name == "unet.head") {
      // evaluated by the head kernel in fp32, weights in file layout [3][C][3][3]
      FFV_TRY(dev_alloc(&L.w_dev, L.w_host.size() * 4, "head weights"));
      FFV_TRY(check(hipMemcpy(L.w_dev, L.w_host.data(), L.w_host.size() * 4, hipMemcpyHostToDevice),
                    "copy head"));
    } else {
      std::vector<uint8_t> packed = pack_layer(L, dt_);
      FFV_TRY(dev_alloc(&L.w_dev, packed.size(), "weights"));
      FFV_TRY(check(hipMemcpy(L.w_dev, packed.data(), packed.size(), hipMemcpyHostToDevice),
                    "copy weights"));
    }
    FFV_TRY(dev_alloc((void**)&L.b_dev, L.b_host.size() * 4, "bias"));
    FFV_TRY(check(hipMemcpy(L.b_dev, L.b_host.data(), L.b_host.size() * 4, hipMemcpyHostToDevice),
                  "copy bias"));
  }
  return Status::ok();
}

CamPlan Net::cam_plan(const Geo& g) const {
  const size_t e = dtype_size(dt_);
  const long P = g.P;
  const int B = base_width_;
  CamPlan c{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  c.X4 = take((size_t)P * 4 * 4);
  c.Xa = take((size_t)P * 8 * e);
  c.L0 = take((size_t)(P / 16) * 4 * 4);
  c.L1 = take((size_t)(P / 4) * 4 * 4);
  const int cw[4] = {B / 2, B, 2 * B, 4 * B};
  for (int k = 0; k < 4; ++k) c.ctx[k] = take((size_t)(P >> (2 * (k + 1))) * cw[k] * e);
  c.bytes = off;
  c.ctmp = align_up((size_t)(P / 4) * (B / 2) * e, 256);
  return c;
}

CamDev Net::cam_dev(const Geo& g, char* block) const {
  CamPlan c = cam_plan(g);
  CamDev d;
  d.X4 = (const float*)(block + c.X4);
  d.L0 = (const float*)(block + c.L0);
  d.L1 = (const float*)(block + c.L1);
  for (int k = 0; k < 4; ++k) d.ctx[k] = block + c.ctx[k];
  return d;
}

ViewPlan Net::view_plan(const Geo& g, int n_view) const {
  const size_t e = dtype_size(dt_);
  const long P = g.P;
  const int B = base_width_;
  ViewPlan p;
  p.g = g;
  p.n_view = n_view;
  const size_t V = n_view;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  p.FM[0] = take(V * (P / 16) * 8 * 4);
  p.FM[1] = take(V * (P / 4) * 8 * 4);
  p.FM[2] = take(V * P * 8 * 4);
  p.I2 = take(V * P * 4 * 4);
  for (int k = 0; k < 4; ++k) p.Fp[k] = take(V * (P >> (2 * (k + 1))) * 4 * 4);
  p.views = take(V * sizeof(ViewDesc));
  const size_t phase0 = off;
  p.xin = take(V * P * 24 * e);
  p.a1 = take(V * (P / 4) * 4 * B * e);
  p.bA = take(V * (P / 16) * 8 * B * e);
  p.bB = take(V * (P / 16) * 8 * B * e);
  const size_t end_vib = off;
  off = phase0;
  p.x0u = take(V * P * 24 * e);
  const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
  for (int k = 0; k < 4; ++k) p.lvl[k] = take(V * (P >> (2 * (k + 1))) * lv_ld[k] * e);
  p.etmp = take(V * (P / 4) * B * e);
  p.u4 = take(V * P * (B / 2) * e);
  p.total = std::max(off, end_vib);
  return p;
}

void Net::drop_graphs() {
  graph_epoch_.fetch_add(1, std::memory_order_acq_rel);
  for (auto& kv : graph_cache_) {
    hipGraphExecDestroy(kv.second.exec);
    for (auto& pe : kv.second.prof) {
      evt_pool_.push_back(pe.a);
      evt_pool_.push_back(pe.b);
    }
  }
  graph_cache_.clear();
}

void Net::add_stat(const PendingEvt& pe) {
  float ms = 0.f;
  hipEventElapsedTime(&ms, pe.a, pe.b);
  KernelStat& ks = stats_[pe.cls];
  ks.launches += 1;
  ks.ms += ms;
  ks.work += pe.work;
}

void Net::set_graphs(bool on) {
  std::lock_guard<std::mutex> lk(call_mu_);
  graphs_ = on;
  if (!on) {
    if (stream_) hipStreamSynchronize(stream_);
    drop_graphs();
  }
}

Status Net::ensure_workspace(size_t bytes) {
  if (bytes <= ws_bytes_) return Status::ok();
  if (ws_) {
    hipStreamSynchronize(stream_);
    drop_graphs();  // they address the old workspace
    hipFree(ws_);
    ws_ = nullptr;
    ws_bytes_ = 0;
  }
  FFV_TRY(dev_alloc(&ws_, bytes, "workspace"));
  ws_bytes_ = bytes;
  return Status::ok();
}

void Net::set_profiling(bool on) {
  ServingPause pause(sched_.get());
  std::lock_guard<std::mutex> lk(call_mu_);
  profiling_ = on;
  stats_.clear();
}

// Record e on x's stream. Under capture the record becomes an event-record
// node of the graph, appended after the nodes captured so far, so the event
// is timestamped on every replay.
void Net::record_event(const Exec& x, hipEvent_t e) {
  if (!x.capture) {
    hipEventRecord(e, x.s);
    return;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  hipGraph_t graph = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t n_deps = 0;
  if (hipStreamGetCaptureInfo_v2(x.s, &cs, &id, &graph, &deps, &n_deps) != hipSuccess ||
      cs != hipStreamCaptureStatusActive) {
    prof_error_ = true;
    return;
  }
  hipGraphNode_t node = nullptr;
  if (hipGraphAddEventRecordNode(&node, graph, deps, n_deps, e) != hipSuccess ||
      hipStreamUpdateCaptureDependencies(x.s, &node, 1, hipStreamSetCaptureDependencies) != hipSuccess)
    prof_error_ = true;
}

void Net::prof_begin(const Exec& x) {
  if (!x.prof) return;
  hipEvent_t e;
  if (!evt_pool_.empty()) {
    e = evt_pool_.back();
    evt_pool_.pop_back();
  } else {
    hipEventCreate(&e);
  }
  record_event(x, e);
  cur_start_ = e;
}

void Net::prof_end(const Exec& x, const char* cls, double work) {
  if (!x.prof || !cur_start_) return;
  hipEvent_t e;
  if (!evt_pool_.empty()) {
    e = evt_pool_.back();
    evt_pool_.pop_back();
  } else {
    hipEventCreate(&e);
  }
  record_event(x, e);
  pending_.push_back({cur_start_, e, cls, work});
  cur_start_ = nullptr;
}

Status Net::kernel_stats(const std::string& name, long* launches, double* ms, double* work) {
  std::lock_guard<std::mutex> lk(call_mu_);
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

namespace {

// Block width (32, 16 or 8) of the halo tiles with the least padded area for
// a launch, or 0 when the halo tiles cannot run it.
int halo_default_width(DType dt, const ConvArgs& a0) {
  int best = 0;
  long best_area = -1;
  for (int tw : {32, 16, 8}) {
    ConvArgs a = a0;
    a.tile_w = tw;
    if (!conv_halo_tile_ok(dt, a)) continue;
    const int th = 256 / tw;
    const long area = (long)((a.Ho + th - 1) / th) * th * ((a.Wo + tw - 1) / tw) * tw;
    if (best_area < 0 || area < best_area) {
      best_area = area;
      best = tw;
    }
  }
  return best;
}

}  // namespace

Status Net::conv(const Exec& x, const Layer& L, const void* in, int in_ld, long in_img_stride,
                 int Hi, int Wi, int n_img, void* out, int out_ld, long out_img_stride,
                 bool out_f32, bool accumulate, bool relu, bool in_fp8, bool out_fp8) {
  ConvArgs a{};
  a.in = in;
  a.in_img_stride = in_img_stride;
  a.in_ld = in_ld;
  a.Hi = Hi;
  a.Wi = Wi;
  a.wgt = in_fp8 ? L.w8_dev : L.w_dev;
  a.w_scale = in_fp8 ? L.w8_scale : nullptr;
  a.out_scale = out_fp8 ? L.out_scale : nullptr;
  a.amax = calibrating_ ? L.amax : nullptr;
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
  a.K_pad = in_fp8 ? round_up(L.K, 128) : L.K_pad;
  a.cout = L.cout;
  a.cout_pad = L.cout_pad;
  a.n_rows = L.rows;
  a.n_img = n_img;
  a.stride = L.transposed ? 1 : L.stride;
  a.transposed = L.mode;
  a.relu = relu ? 1 : 0;
  a.out_f32 = out_f32 ? 1 : 0;
  a.accumulate = accumulate ? 1 : 0;
  a.taps = L.mode == 1 ? 4 : 9;
  a.zero = zero_;
  a.tile_w = conv_tile_width(a.Ho, a.Wo);
  ConvTile tile = L.tile;
  const DType kdt = in_fp8 ? DType::FP8 : dt_;
  // few output channels over a stride-1 3x3 neighbourhood: the persistent
  // kernel with resident weights where they fit, else the halo kernel
  if (L.rows <= 64 && conv_resident_ok(kdt, a, L.rows <= 32 ? 32 : 64)) {
    tile = L.rows <= 32 ? ConvTile::R32 : ConvTile::R64;
    a.tile_w = 16;
  } else if (L.rows <= 32 && conv_halo_ok(kdt, a)) {
    tile = ConvTile::H32;
    a.tile_w = 16;
  } else if (!L.transposed && kdt != DType::F32 && L.rows > 128 && halo_default_width(kdt, a) > 0) {
    // 3x3 stride-1 convs with more than 128 outputs (the 256-channel chains):
    // the two-group halo tile, the fastest tile for them when tuned, at the
    // least padded block width it accepts
    tile = ConvTile::P256;
    a.tile_w = halo_default_width(kdt, a);
  } else if (!L.transposed && !out_f32 && L.rows <= 128) {
    // convs over a few input channels (8 to 32): the persistent kernel with
    // resident weights, narrowest N tile that holds the layer
    const int bn = L.rows <= 32 ? 32 : (L.rows <= 64 ? 64 : 128);
    if (conv_resident_s2_ok(kdt, a, bn)) {
      tile = bn == 32 ? ConvTile::S32 : (bn == 64 ? ConvTile::S64 : ConvTile::S128);
      a.tile_w = 16;
    }
  }
  if (!tuned_.empty() || recording_) {
    const TuneKey key{L.name, in_fp8 ? 1 : 0, a.Ho, a.Wo, n_img};
    auto it = tuned_.find(key);
    if (it != tuned_.end()) {
      tile = it->second.tile;
      a.tile_w = it->second.tile_w;
    }
    if (recording_) recs_.push_back(TuneRec{key, a, kdt});
  }
  if (in_ld < L.cin_pad || in_ld % (in_fp8 ? 16 : 8) != 0) return Status::err(-4, "conv input stride");
  if ((in_fp8 && !L.w8_dev) || (out_fp8 && !L.out_scale)) return Status::err(-7, "fp8 layer not quantised");
  const double flops = 2.0 * n_img * (double)a.Hout * a.Wout * L.cout * L.cin *
                       (L.transposed ? 4.0 : 9.0);
  const char* cls = L.transposed ? "convT"
                                 : ((L.cin == 8 * base_width_ && L.cout == 8 * base_width_ &&
                                     L.stride == 1)
                                        ? "conv256"
                                        : "conv");
  if (x.n_groups > 1) {
    // views of several sizes: one launch over the size groups, each group's
    // images at its own size (a shift of the plan's size: every level is the
    // padded size over a power of two) and at its offset in the buffers
    int k = 0;
    while (k < 8 && (x.plan_hp >> k) > Hi) ++k;
    if ((x.plan_hp >> k) != Hi) return Status::err(-4, "grouped conv: level size");
    int n_total = 0;
    for (int j = 0; j < x.n_groups; ++j) n_total += x.groups[j].n;
    if (n_total != n_img || x.n_groups > ConvGroup::kMax) return Status::err(-4, "grouped conv: groups");
    // tiles without a grouped form (the persistent kernels, the one-group
    // halo tiles): the generic tile of the same N width
    ConvTile gt = tile;
    if (!conv_tile_groupable(gt)) {
      const int bn = conv_tile_bn(gt);
      gt = bn == 32 ? ConvTile::N32 : (bn == 64 ? ConvTile::N64 : (bn == 128 ? ConvTile::N128 : ConvTile::N256));
    }
    bool halo_tile = gt == ConvTile::P256;
    const size_t in_e = in_fp8 ? 1 : dtype_size(dt_);
    const size_t out_e = out_f32 ? 4 : (out_fp8 ? 1 : dtype_size(dt_));
    ConvArgs g[ConvGroup::kMax];
    double gflops = 0.0;
    for (int j = 0; j < x.n_groups; ++j) {
      const ViewGroup& vg = x.groups[j];
      ConvArgs& b = g[j];
      b = a;
      b.n_img = vg.n;
      b.Hi = vg.Hp >> k;
      b.Wi = vg.Wp >> k;
      if (L.transposed) {
        b.Ho = b.Hi;
        b.Wo = b.Wi;
        b.Hout = 2 * b.Hi;
        b.Wout = 2 * b.Wi;
      } else {
        b.Ho = (b.Hi - 1) / L.stride + 1;
        b.Wo = (b.Wi - 1) / L.stride + 1;
        b.Hout = b.Ho;
        b.Wout = b.Wo;
      }
      b.in = static_cast<const char*>(in) + (size_t)vg.first * in_img_stride * in_e;
      b.out = static_cast<char*>(out) + (size_t)vg.first * out_img_stride * out_e;
      b.tile_w = halo_tile ? halo_default_width(kdt, b) : conv_tile_width(b.Ho, b.Wo);
      if (b.tile_w == 0) {
        // the halo tiles cannot take this group: the generic tile of the same
        // N width for every group (restart; the generic tile takes any width)
        gt = conv_tile_bn(gt) == 256 ? ConvTile::N256 : ConvTile::N128;
        halo_tile = false;
        j = -1;
        gflops = 0.0;
        continue;
      }
      gflops += 2.0 * vg.n * (double)b.Hout * b.Wout * L.cout * L.cin * (L.transposed ? 4.0 : 9.0);
    }
    prof_begin(x);
    Status st = check(launch_conv_grouped(kdt, gt, g, x.n_groups, x.s), L.name.c_str());
    prof_end(x, cls, gflops);
    return st;
  }
  prof_begin(x);
  Status st = check(launch_conv(kdt, tile, a, x.s), L.name.c_str());
  prof_end(x, cls, flops);
  return st;
}

Status Net::build_cameras(const Exec& x, const Geo& g, const float* const* src_dev, int n_cam,
                          char* const* blocks, char* ctmp, bool context) {
  if (n_cam <= 0) return Status::ok();
  const CamPlan c = cam_plan(g);
  const int B = base_width_;
  // Camera blocks of one call are contiguous and equally spaced, so every
  // per-camera pass runs as one batched launch over them.
  const long stride = blocks[n_cam - 1] - blocks[0];
  const long cs = n_cam > 1 ? stride / (n_cam - 1) : (long)c.bytes;
  for (int i = 1; i < n_cam; ++i)
    if (blocks[i] - blocks[0] != i * cs) return Status::err(-4, "camera blocks not equally spaced");
  const size_t e = dtype_size(dt_);
  if (cs % 256 != 0) return Status::err(-4, "camera stride");
  char* b0 = blocks[0];
  const long P = g.P;
  // ingest, padding and the image pyramid, one camera per launch
  for (int i = 0; i < n_cam; ++i) {
    prof_begin(x);
    FFV_TRY(check(launch_ingest(src_dev + i, 1, g.H, g.W, g.Hp, g.Wp, (float*)(blocks[i] + c.X4),
                                blocks[i] + c.Xa, dt_, x.s),
                  "ingest"));
    FFV_TRY(check(launch_resample4((const float*)(blocks[i] + c.X4), 1, g.Hp, g.Wp,
                                   (float*)(blocks[i] + c.L0), g.Hp / 4, g.Wp / 4, x.s),
                  "resample L0"));
    FFV_TRY(check(launch_resample4((const float*)(blocks[i] + c.X4), 1, g.Hp, g.Wp,
                                   (float*)(blocks[i] + c.L1), g.Hp / 2, g.Wp / 2, x.s),
                  "resample L1"));
    prof_end(x, "pixel", (double)g.H * g.W * 12 + P * (16.0 + 8 * e) + 2 * P * 16.0 +
                             (P / 16 + P / 4) * 16.0);
  }
  if (!context) return Status::ok();
  // ContextNet batched over the cameras: image stride = camera block stride
  const int cw[4] = {B / 2, B, 2 * B, 4 * B};
  const char* src = b0 + c.Xa;
  long src_stride_el = cs / (long)e;
  int src_ld = 8, h = g.Hp, w = g.Wp;
  for (int k = 0; k < 4; ++k) {
    const int ho = h / 2, wo = w / 2;
    char n1[32], n2[32];
    snprintf(n1, sizeof n1, "ctx.conv%d", 2 * k + 1);
    snprintf(n2, sizeof n2, "ctx.conv%d", 2 * k + 2);
    const long tmp_stride = (long)(c.ctmp / e);
    FFV_TRY(conv(x, layer(n1), src, src_ld, src_stride_el, h, w, n_cam, ctmp, cw[k], tmp_stride, false,
                 false, true));
    FFV_TRY(conv(x, layer(n2), ctmp, cw[k], tmp_stride, ho, wo, n_cam, b0 + c.ctx[k], cw[k],
                 src_stride_el, false, false, true));
    src = b0 + c.ctx[k];
    src_ld = cw[k];
    h = ho;
    w = wo;
  }
  return Status::ok();
}

Status Net::run_views(const Exec& x, const ViewPlan& p, const CamDev* cams,
                      const ViewDesc* views_in, int nv, bool views_on_device, bool refine) {
  const Geo& g = p.g;
  const long P = g.P;
  const int B = base_width_;
  const size_t e = dtype_size(dt_);
  const ViewDesc* views = views_in;
  if (!views_on_device) {
    ViewDesc* slot = (ViewDesc*)x.at(p.views);
    FFV_TRY(check(hipMemcpyAsync(slot, views_in, sizeof(ViewDesc) * nv, hipMemcpyHostToDevice, x.s),
                  "copy views"));
    views = slot;
  }
  const int tp = t_plane_ ? 1 : 0;

  // stage 0 input
  const int h0 = g.Hp / 4, w0 = g.Wp / 4;
  prof_begin(x);
  FFV_TRY(check(launch_assemble0(views, nv, cams, h0, w0, x.at(p.xin), 8, dt_, tp, x.s), "assemble0"));
  prof_end(x, "pixel", (double)nv * (P / 16) * (32.0 + 8 * e));

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
      prof_begin(x);
      FFV_TRY(check(launch_transition(views, nv, cams, s, (const float*)x.at(p.FM[s - 1]), h / 2, w / 2,
                                      h, w, x.at(p.xin), 24, (float*)x.at(p.FM[s]), dt_, tp, x.s),
                    "transition"));
      prof_end(x, "pixel", (double)nv * Ps * (20.0 / 4 + 16 * 4 + 24 * e + 32));
    }
    const int h1 = h / 2, w1 = w / 2, h2 = h / 4, w2 = w / 4;
    const int C1 = 4 * B, C2 = 8 * B;
    // FP8 nets keep the VIBlock's inner activations (a1, the 256-channel
    // chain, a9) in fp8; conv1 quantises its output, convT2 reads fp8.
    const bool q = vib_fp8();
    FFV_TRY(conv(x, L("conv1"), x.at(p.xin), in_ld, Ps * in_ld, h, w, nv, x.at(p.a1), C1,
                 (long)h1 * w1 * C1, false, false, true, false, q));
    FFV_TRY(conv(x, L("conv2"), x.at(p.a1), C1, (long)h1 * w1 * C1, h1, w1, nv, x.at(p.bA), C2,
                 (long)h2 * w2 * C2, false, false, true, q, q));
    void* cur = x.at(p.bA);
    void* nxt = x.at(p.bB);
    for (int i = 3; i <= 8; ++i) {
      char suf[16];
      snprintf(suf, sizeof suf, "conv%d", i);
      FFV_TRY(conv(x, L(suf), cur, C2, (long)h2 * w2 * C2, h2, w2, nv, nxt, C2, (long)h2 * w2 * C2,
                   false, false, true, q, q));
      std::swap(cur, nxt);
    }
    FFV_TRY(conv(x, L("convT1"), cur, C2, (long)h2 * w2 * C2, h2, w2, nv, x.at(p.a1), C1,
                 (long)h1 * w1 * C1, false, false, true, q, q));
    FFV_TRY(conv(x, L("convT2"), x.at(p.a1), C1, (long)h1 * w1 * C1, h1, w1, nv, x.at(p.FM[s]), 8,
                 Ps * 8, true, s > 0, false, q, false));
  }

  // final warp + blend, U-Net input
  prof_begin(x);
  FFV_TRY(check(launch_final(views, nv, cams, (const float*)x.at(p.FM[2]), g.Hp, g.Wp,
                             (float*)x.at(p.I2), x.at(p.x0u), 24, dt_, x.s),
                "final"));
  prof_end(x, "pixel", (double)nv * P * (20.0 + 16 * 4 + 16 + 24 * e));

  if (!refine) {  // the blend is the output
    prof_begin(x);
    FFV_TRY(check(launch_blend_out((const float*)x.at(p.I2), views, nv, g.Hp, g.Wp, g.H, g.W, x.s),
                  "blend out"));
    prof_end(x, "pixel", (double)nv * (16.0 * g.H * g.W + 12.0 * g.H * g.W));
    return Status::ok();
  }

  // flow pyramid and context warps
  {
    const float* src = (const float*)x.at(p.FM[2]);
    int ld = 8, h = g.Hp, w = g.Wp;
    const int cw[4] = {B / 2, B, 2 * B, 4 * B};
    const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
    const int lv_off[4] = {2 * B, 4 * B, 8 * B, 8 * B};
    for (int k = 0; k < 4; ++k) {
      const int ho = h / 2, wo = w / 2;
      const long Pk = (long)ho * wo;
      prof_begin(x);
      FFV_TRY(check(launch_flow_down(src, ld, views, nv, k, h, w, (float*)x.at(p.Fp[k]), x.s), "flow_down"));
      FFV_TRY(check(launch_ctx_warp(views, nv, cams, k, cw[k], (const float*)x.at(p.Fp[k]), ho, wo,
                                    x.at(p.lvl[k]) + lv_off[k] * e, lv_ld[k], Pk * lv_ld[k], dt_, x.s),
                    "ctx_warp"));
      prof_end(x, "pixel", (double)nv * ((double)h * w * 16 + Pk * 16 + 2 * Pk * 16 +
                                         2.0 * Pk * cw[k] * e * 2));
      src = (const float*)x.at(p.Fp[k]);
      ld = 4;
      h = ho;
      w = wo;
    }
  }

  // context-aware U-Net
  {
    const int ew[4] = {B, 2 * B, 4 * B, 8 * B};
    const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
    const void* src = x.at(p.x0u);
    int src_ld = 24, h = g.Hp, w = g.Wp;
    for (int k = 0; k < 4; ++k) {
      const int ho = h / 2, wo = w / 2;
      char n1[32], n2[32];
      snprintf(n1, sizeof n1, "unet.enc%d", 2 * k + 1);
      snprintf(n2, sizeof n2, "unet.enc%d", 2 * k + 2);
      FFV_TRY(conv(x, layer(n1), src, src_ld, (long)h * w * src_ld, h, w, nv, x.at(p.etmp), ew[k],
                   (long)ho * wo * ew[k], false, false, true));
      // level buffer k holds [u | d | wc_l | wc_r]; d_{k+1} follows the decoder slot
      const int d_off = k < 3 ? ew[k] : 0;
      char* dst = x.at(p.lvl[k]) + (size_t)d_off * e;
      FFV_TRY(conv(x, layer(n2), x.at(p.etmp), ew[k], (long)ho * wo * ew[k], ho, wo, nv, dst, lv_ld[k],
                   (long)ho * wo * lv_ld[k], false, false, true));
      src = dst;
      src_ld = lv_ld[k];
      h = ho;
      w = wo;
    }
    for (int k = 0; k < 4; ++k) {
      const int lvl_in = 3 - k;
      const int hi = g.Hp >> (lvl_in + 1), wi = g.Wp >> (lvl_in + 1);
      char nm[32];
      snprintf(nm, sizeof nm, "unet.dec%d", k + 1);
      void* dst;
      int dst_ld;
      if (k < 3) {
        dst = x.at(p.lvl[lvl_in - 1]);
        dst_ld = lv_ld[lvl_in - 1];
      } else {
        dst = x.at(p.u4);
        dst_ld = B / 2;
      }
      FFV_TRY(conv(x, layer(nm), x.at(p.lvl[lvl_in]), lv_ld[lvl_in], (long)hi * wi * lv_ld[lvl_in], hi,
                   wi, nv, dst, dst_ld, (long)(2 * hi) * (2 * wi) * dst_ld, false, false, true));
    }
  }

  // output head
  {
    const Layer& Hd = layer("unet.head");
    prof_begin(x);
    FFV_TRY(check(launch_head(x.at(p.u4), B / 2, B / 2, (const float*)Hd.w_dev, Hd.b_dev,
                              (const float*)x.at(p.I2), views, nv, g.Hp, g.Wp, g.H, g.W, dt_, x.s),
                  "head"));
    prof_end(x, "head", (double)nv * ((double)P * (B / 2) * e + (double)P * 16 + 12.0 * g.H * g.W));
  }
  return Status::ok();
}

Status Net::interpolate(const float* const* left, const float* const* right, int n_pairs, int H,
                        int W, const float* t, int n_t, float* out) {
  std::lock_guard<std::mutex> lk(call_mu_);
  return interpolate_locked(left, right, n_pairs, H, W, t, n_t, out);
}

Status Net::interpolate_blend(const float* const* left, const float* const* right, int n_pairs, int H,
                              int W, const float* t, int n_t, float* out) {
  std::lock_guard<std::mutex> lk(call_mu_);
  std::vector<float*> outs((size_t)n_pairs * n_t);
  for (size_t v = 0; v < outs.size(); ++v) outs[v] = out + v * 3 * (size_t)H * W;
  return run_call(left, right, n_pairs, H, W, t, n_t, outs.data(), false);
}

Status Net::interpolate_recursive(const float* const* left, const float* const* right, int n_pairs,
                                  int H, int W, int levels, float* out) {
  if (levels < 1 || levels > 10) return Status::err(-1, "levels must lie in [1, 10]");
  std::lock_guard<std::mutex> lk(call_mu_);
  const int n = 1 << levels;
  const size_t img = 3 * (size_t)H * W;
  auto view = [&](int i, int k) -> float* { return out + ((size_t)i * (n - 1) + (k - 1)) * img; };
  const float half = 0.5f;
  for (int level = 1; level <= levels; ++level) {
    const int step = n >> level;
    std::vector<const float*> l, r;
    std::vector<float*> o;
    for (int i = 0; i < n_pairs; ++i)
      for (int k = step; k < n; k += 2 * step) {
        l.push_back(k - step == 0 ? left[i] : view(i, k - step));
        r.push_back(k + step == n ? right[i] : view(i, k + step));
        o.push_back(view(i, k));
      }
    FFV_TRY(run_call(l.data(), r.data(), (int)l.size(), H, W, &half, 1, o.data(), true));
  }
  return Status::ok();
}

Status Net::interpolate_locked(const float* const* left, const float* const* right, int n_pairs,
                               int H, int W, const float* t, int n_t, float* out) {
  std::vector<float*> outs((size_t)n_pairs * n_t);
  for (size_t v = 0; v < outs.size(); ++v) outs[v] = out + v * 3 * (size_t)H * W;
  return run_call(left, right, n_pairs, H, W, t, n_t, outs.data(), true);
}

Status Net::run_call(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                     const float* t, int n_t, float* const* outs, bool refine) {
  if (!ready() && !calibrating_) return Status::err(-7, "FP8 net needs ffv_calibrate first");
  FFV_TRY(check(hipSetDevice(device_), "hipSetDevice"));
  const Geo g = Geo::of(H, W);

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

  // workspace: [camera blocks][camera scratch][camera table + image table][views]
  const CamPlan cp = cam_plan(g);
  const size_t cam_region = align_up(cp.bytes * n_cam, 256);
  const size_t ctmp_region = align_up(cp.ctmp * n_cam, 256);
  const size_t tab_region = align_up(sizeof(CamDev) * n_cam + sizeof(void*) * n_cam, 256) +
                            align_up(sizeof(ViewDesc) * n_view_total, 256);
  const size_t fixed = cam_region + ctmp_region + tab_region;
  const size_t per_view = view_plan(g, 2).total - view_plan(g, 1).total;
  int chunk = n_view_total;
  if (!debug_ && fixed + view_plan(g, chunk).total > ws_cap_)
    chunk = (int)std::max<size_t>(1, ws_cap_ > fixed + per_view ? (ws_cap_ - fixed) / per_view : 1);
  chunk = std::max(1, std::min(chunk, n_view_total));
  while (chunk > 1 && fixed + view_plan(g, chunk).total > ws_cap_) --chunk;
  const ViewPlan vp = view_plan(g, chunk);
  FFV_TRY(ensure_workspace(fixed + vp.total));

  char* base = (char*)ws_;
  Exec x;
  x.s = stream_;
  x.prof = profiling_;
  std::vector<char*> blocks(n_cam);
  std::vector<CamDev> camdev(n_cam);
  for (int i = 0; i < n_cam; ++i) {
    blocks[i] = base + cp.bytes * i;
    camdev[i] = cam_dev(g, blocks[i]);
  }
  char* ctmp = base + cam_region;
  CamDev* cam_tab = (CamDev*)(base + cam_region + ctmp_region);
  const float** src_tab = (const float**)((char*)cam_tab + sizeof(CamDev) * n_cam);
  FFV_TRY(check(hipMemcpyAsync(cam_tab, camdev.data(), sizeof(CamDev) * n_cam, hipMemcpyHostToDevice,
                               stream_),
                "copy camera table"));
  FFV_TRY(check(hipMemcpyAsync(src_tab, cams.data(), sizeof(void*) * n_cam, hipMemcpyHostToDevice,
                               stream_),
                "copy image table"));

  std::vector<ViewDesc> vd(n_view_total);
  for (int i = 0; i < n_pairs; ++i)
    for (int j = 0; j < n_t; ++j) {
      ViewDesc& d = vd[(size_t)i * n_t + j];
      d = ViewDesc{};
      d.cam_l = li[i];
      d.cam_r = ri[i];
      d.t = t[j];
      d.out = outs[(size_t)i * n_t + j];
      d.hp = g.Hp;
      d.wp = g.Wp;
      d.h = g.H;
      d.w = g.W;
    }
  // Graph replay needs every per-call value in device tables: the camera
  // and image tables above, and here all views' descriptors.
  const bool use_graph = graphs_ && !debug_ && !calibrating_ && !recording_;
  ViewDesc* view_tab = (ViewDesc*)(base + cam_region + ctmp_region +
                                   align_up(sizeof(CamDev) * n_cam + sizeof(void*) * n_cam, 256));
  if (use_graph)
    FFV_TRY(check(hipMemcpyAsync(view_tab, vd.data(), sizeof(ViewDesc) * n_view_total,
                                 hipMemcpyHostToDevice, stream_),
                  "copy view table"));
  x.capture = use_graph;
  Exec xv = x;
  xv.ws = base + fixed;
  auto launch_all = [&]() -> Status {
    FFV_TRY(build_cameras(x, g, src_tab, n_cam, blocks.data(), ctmp, refine));
    for (int v0 = 0; v0 < n_view_total; v0 += chunk) {
      const int nv = std::min(chunk, n_view_total - v0);
      FFV_TRY(run_views(xv, vp, cam_tab, use_graph ? view_tab + v0 : vd.data() + v0, nv, use_graph,
                        refine));
    }
    return Status::ok();
  };
  const GraphEntry* ran = nullptr;
  if (use_graph) {
    const GraphKey key{H, W, n_cam, n_view_total, chunk, ws_, vib_fp8(), profiling_, refine};
    auto it = graph_cache_.find(key);
    if (it == graph_cache_.end()) {
      pending_.clear();
      FFV_TRY(check(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal), "begin capture"));
      prof_error_ = false;
      Status st = launch_all();
      if (st.good() && prof_error_) st = Status::err(-4, "profiling: event-record node in graph capture");
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(stream_, &graph);
      GraphEntry entry;
      entry.prof = std::move(pending_);
      pending_.clear();
      if (!st.good() || ec != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        for (auto& pe : entry.prof) {
          evt_pool_.push_back(pe.a);
          evt_pool_.push_back(pe.b);
        }
        FFV_TRY(st);
        return check(ec, "end capture");
      }
      const hipError_t ei = hipGraphInstantiate(&entry.exec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        for (auto& pe : entry.prof) {
          evt_pool_.push_back(pe.a);
          evt_pool_.push_back(pe.b);
        }
        return check(ei, "graph instantiate");
      }
      if (graph_cache_.size() >= 64) {
        FFV_TRY(check(hipStreamSynchronize(stream_), "hipStreamSynchronize"));
        drop_graphs();
      }
      it = graph_cache_.emplace(key, std::move(entry)).first;
    }
    FFV_TRY(check(hipGraphLaunch(it->second.exec, stream_), "graph launch"));
    ran = &it->second;
  } else {
    FFV_TRY(launch_all());
  }
  FFV_TRY(check(hipStreamSynchronize(stream_), "hipStreamSynchronize"));
  last_plan_ = vp;
  last_views_ws_ = xv.ws;
  last_cam_l_ = blocks[li[0]];
  last_cam_r_ = blocks[ri[0]];
  have_taps_ = true;
  if (profiling_) {
    if (ran)
      for (const auto& pe : ran->prof) add_stat(pe);
    for (auto& pe : pending_) {
      add_stat(pe);
      evt_pool_.push_back(pe.a);
      evt_pool_.push_back(pe.b);
    }
    pending_.clear();
  }
  return Status::ok();
}

Status Net::debug_tap(const std::string& name, float* dst, size_t cap, int dims[3]) {
  std::lock_guard<std::mutex> lk(call_mu_);
  if (!have_taps_) return Status::err(-7, "no forward pass recorded");
  const ViewPlan& p = last_plan_;
  const Geo& g = p.g;
  const int B = base_width_;
  const char* src = nullptr;
  DType dt = dt_;
  int C = 0, ld = 0, h = 0, w = 0;
  // level k (1..4) of a tap name ending in a digit
  const int k = name.empty() ? 0 : name.back() - '0';
  const bool lvl_ok = k >= 1 && k <= 4;
  const std::string stem = name.substr(0, name.size() - 1);
  const int lv_ld[4] = {3 * B, 6 * B, 12 * B, 16 * B};
  const int cw[4] = {B / 2, B, 2 * B, 4 * B};
  if (name == "F0" || name == "F1" || name == "F2") {
    const int s = name[1] - '0';
    h = g.Hp * (1 << s) / 4;
    w = g.Wp * (1 << s) / 4;
    src = last_views_ws_ + p.FM[s];
    C = 5;
    ld = 8;
    dt = DType::F32;
  } else if (name == "I2") {
    h = g.Hp;
    w = g.Wp;
    src = last_views_ws_ + p.I2;
    C = 3;
    ld = 4;
    dt = DType::F32;
  } else if (name == "x0") {  // U-Net input [X_l, X_r, W_l, W_r, M, F]
    h = g.Hp;
    w = g.Wp;
    src = last_views_ws_ + p.x0u;
    C = 17;
    ld = 24;
  } else if (lvl_ok && (stem == "d" || stem == "u" || stem == "wcl" || stem == "wcr")) {
    // U-Net level buffer k - 1 holds [u | d | wc_l | wc_r] at 2^-k of the
    // padded size (the deepest: [d4 | wc_l | wc_r]); u4 has its own buffer
    h = g.Hp >> k;
    w = g.Wp >> k;
    const int e = (int)dtype_size(dt_);
    const int enc_w = B << (k - 1);  // d_k channels
    const char* lvl = last_views_ws_ + p.lvl[k - 1];
    ld = lv_ld[k - 1];
    if (stem == "d") {
      src = lvl + (size_t)(k < 4 ? enc_w : 0) * e;
      C = enc_w;
    } else if (stem == "u") {
      C = (16 * B) >> (k + 1);  // 4B, 2B, B, B/2
      if (k == 4) {
        h = g.Hp;
        w = g.Wp;
        src = last_views_ws_ + p.u4;
        ld = B / 2;
      } else {
        // u_k sits in the u slot of level buffer 3 - k, at twice its size
        h = g.Hp >> (4 - k);
        w = g.Wp >> (4 - k);
        src = last_views_ws_ + p.lvl[3 - k];
        ld = lv_ld[3 - k];
      }
    } else {
      const int off = k < 4 ? 2 * enc_w : enc_w;
      src = lvl + (size_t)(off + (stem == "wcr" ? cw[k - 1] : 0)) * e;
      C = cw[k - 1];
    }
  } else if (lvl_ok && (stem == "cl" || stem == "cr")) {  // context features of either camera
    const CamPlan c = cam_plan(g);
    h = g.Hp >> k;
    w = g.Wp >> k;
    src = (stem == "cl" ? last_cam_l_ : last_cam_r_) + c.ctx[k - 1];
    C = cw[k - 1];
    ld = C;
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

// VIBlock layers in execution order; each reads the previous one's output.
static std::vector<std::string> vib_chain(int s) {
  std::vector<std::string> v;
  for (const char* n : {"conv1", "conv2", "conv3", "conv4", "conv5", "conv6", "conv7", "conv8", "convT1",
                        "convT2"})
    v.push_back("vib" + std::to_string(s) + "." + n);
  return v;
}

Status Net::calibrate(const float* left, const float* right, int H, int W, float t) {
  if (!fp8_) return Status::err(-7, "calibration applies to FP8 nets");
  // served batches read the fp8 weights and scales this call rewrites
  ServingPause pause(sched_.get());
  std::lock_guard<std::mutex> lk(call_mu_);
  FFV_TRY(check(hipSetDevice(device_), "hipSetDevice"));
  for (int s = 0; s < 3; ++s)
    for (const std::string& nm : vib_chain(s)) {
      Layer& L = layers_.at(nm);
      if (!L.amax) FFV_TRY(check(hipMalloc((void**)&L.amax, sizeof(float) * L.cout), "hipMalloc amax"));
      FFV_TRY(check(hipMemsetAsync(L.amax, 0, sizeof(float) * L.cout, stream_), "zero amax"));
    }
  float* out = nullptr;
  FFV_TRY(check(hipMalloc((void**)&out, sizeof(float) * 3 * (size_t)H * W), "hipMalloc"));
  calibrating_ = true;
  Status st = interpolate_locked(&left, &right, 1, H, W, &t, 1, out);
  calibrating_ = false;
  hipFree(out);
  FFV_TRY(st);
  for (int s = 0; s < 3; ++s)
    for (const std::string& nm : vib_chain(s)) {
      Layer& L = layers_.at(nm);
      std::vector<float> amax(L.cout);
      FFV_TRY(check(hipMemcpy(amax.data(), L.amax, sizeof(float) * L.cout, hipMemcpyDeviceToHost),
                    "read amax"));
      L.act_scale.resize(L.cout);
      for (int o = 0; o < L.cout; ++o) L.act_scale[o] = std::max(amax[o], 1e-6f) / 448.f;
    }
  FFV_TRY(quantize_vib_layers());
  calibrated_ = true;
  drop_graphs();  // captured with the previous weights and scales
  return Status::ok();
}

// Quantise the VIBlock layers that read fp8 activations: the producer's
// per-channel activation scale is folded into the weights, then each output
// channel gets its own weight scale (max |w'| / 448). Producers get their
// output quantisation scale 1 / activation scale.
Status Net::quantize_vib_layers() {
  for (int s = 0; s < 3; ++s) {
    const std::vector<std::string> chain = vib_chain(s);
    for (size_t li = 0; li < chain.size(); ++li) {
      Layer& L = layers_.at(chain[li]);
      if (li + 1 < chain.size()) {
        std::vector<float> inv(L.cout);
        for (int o = 0; o < L.cout; ++o) inv[o] = 1.f / L.act_scale[o];
        if (!L.out_scale)
          FFV_TRY(check(hipMalloc((void**)&L.out_scale, sizeof(float) * L.cout), "hipMalloc scale"));
        FFV_TRY(check(hipMemcpy(L.out_scale, inv.data(), sizeof(float) * L.cout, hipMemcpyHostToDevice),
                      "copy scale"));
      }
      if (li == 0) continue;  // conv1 reads the bf16 stage input
      const Layer& P = layers_.at(chain[li - 1]);
      std::vector<float> w = L.w_host;
      const int taps = L.transposed ? 16 : 9;
      // fold the input channel scale: conv [o][c][t], transposed [c][o][t]
      for (int c = 0; c < L.cin; ++c)
        for (int o = 0; o < L.cout; ++o)
          for (int k = 0; k < taps; ++k) {
            const size_t idx = L.transposed ? ((size_t)c * L.cout + o) * taps + k
                                            : ((size_t)o * L.cin + c) * taps + k;
            w[idx] *= P.act_scale[c];
          }
      std::vector<float> ws(L.cout, 0.f);
      for (int c = 0; c < L.cin; ++c)
        for (int o = 0; o < L.cout; ++o)
          for (int k = 0; k < taps; ++k) {
            const size_t idx = L.transposed ? ((size_t)c * L.cout + o) * taps + k
                                            : ((size_t)o * L.cin + c) * taps + k;
            ws[o] = std::max(ws[o], std::fabs(w[idx]));
          }
      for (int o = 0; o < L.cout; ++o) ws[o] = std::max(ws[o], 1e-30f) / 448.f;
      for (int c = 0; c < L.cin; ++c)
        for (int o = 0; o < L.cout; ++o)
          for (int k = 0; k < taps; ++k) {
            const size_t idx = L.transposed ? ((size_t)c * L.cout + o) * taps + k
                                            : ((size_t)o * L.cin + c) * taps + k;
            w[idx] /= ws[o];
          }
      const int k_pad = round_up(L.K, 128);
      std::vector<float> pf = pack_layer_f(L, conv_k_step(DType::FP8), k_pad, w);
      std::vector<uint8_t> q(pf.size());
      for (size_t i = 0; i < pf.size(); ++i) q[i] = f2f8(pf[i]);
      if (!L.w8_dev) FFV_TRY(check(hipMalloc(&L.w8_dev, q.size()), "hipMalloc fp8 weights"));
      FFV_TRY(check(hipMemcpy(L.w8_dev, q.data(), q.size(), hipMemcpyHostToDevice), "copy fp8 weights"));
      if (!L.w8_scale)
        FFV_TRY(check(hipMalloc((void**)&L.w8_scale, sizeof(float) * L.cout), "hipMalloc w scale"));
      FFV_TRY(check(hipMemcpy(L.w8_scale, ws.data(), sizeof(float) * L.cout, hipMemcpyHostToDevice),
                    "copy w scale"));
    }
  }
  return Status::ok();
}

Status Net::autotune(const float* const* left, const float* const* right, int n_pairs, int H, int W,
                     const float* t, int n_t, float* out, int* n_tuned) {
  if (n_tuned) *n_tuned = 0;
  // no served batch may run while launches are recorded and re-timed
  ServingPause pause(sched_.get());
  // 1. run the call once, recording every conv launch (eager, so each
  //    launch passes through conv()); its output is the call's result
  std::lock_guard<std::mutex> lk(call_mu_);
  recs_.clear();
  recording_ = true;
  Status st = interpolate_locked(left, right, n_pairs, H, W, t, n_t, out);
  recording_ = false;
  FFV_TRY(st);
  // 2. re-run each recorded launch with every candidate tile shape. The
  //    launches read and write only the workspace, whose contents are dead
  //    once the call has returned, and conv kernels address memory from
  //    their shapes alone, whatever values they meet.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  FFV_TRY(check(hipEventCreate(&e0), "hipEventCreate"));
  Status res = check(hipEventCreate(&e1), "hipEventCreate");
  std::map<TuneKey, TuneVal> found;
  const ConvTile tiles[14] = {ConvTile::N256, ConvTile::N128, ConvTile::N64,  ConvTile::N32, ConvTile::H32,
                              ConvTile::H256, ConvTile::H128, ConvTile::R32,  ConvTile::R64, ConvTile::S32,
                              ConvTile::S64,  ConvTile::S128, ConvTile::Q256, ConvTile::P256};
  const int widths[4] = {8, 16, 32, 64};
  for (size_t r = 0; res.good() && r < recs_.size(); ++r) {
    const TuneRec& rec = recs_[r];
    if (found.count(rec.key)) continue;
    const int rows32 = round_up(rec.a.n_rows, 32);
    long min_area = -1;
    for (int tw : widths) {
      const int th = 256 / tw;
      const long area = (long)((rec.a.Ho + th - 1) / th) * th * ((rec.a.Wo + tw - 1) / tw) * tw;
      if (min_area < 0 || area < min_area) min_area = area;
    }
    float best_ms = -1.f;
    TuneVal best{};
    for (int ti = 0; res.good() && ti < 14; ++ti) {
      const bool resident = tiles[ti] == ConvTile::R32 || tiles[ti] == ConvTile::R64;
      const bool s2 = tiles[ti] == ConvTile::S32 || tiles[ti] == ConvTile::S64 || tiles[ti] == ConvTile::S128;
      const bool halo = tiles[ti] == ConvTile::H32 || resident || s2;
      const bool halo_big = tiles[ti] == ConvTile::H256 || tiles[ti] == ConvTile::H128 || tiles[ti] == ConvTile::Q256 ||
                            tiles[ti] == ConvTile::P256;
      const int bn = conv_tile_bn(tiles[ti]);
      // at least half of every tile's columns real (a 256-column halo tile
      // over a per-phase transposed conv holds two, or with 2 x 4 waves
      // four, phases)
      const bool halo256 = tiles[ti] == ConvTile::H256 || tiles[ti] == ConvTile::P256;
      const bool paired = rec.a.transposed == 1 && ((halo256 && rows32 <= 128) ||
                                                    (tiles[ti] == ConvTile::Q256 && rows32 <= 64));
      if (bn >= 2 * rows32 && !paired) continue;
      // the 2 x 4-wave layout only where it groups four phases
      if (tiles[ti] == ConvTile::Q256 && !(rec.a.transposed == 1 && rows32 <= 64)) continue;
      if (tiles[ti] == ConvTile::H32 && !conv_halo_ok(rec.dt, rec.a)) continue;
      if (resident && !conv_resident_ok(rec.dt, rec.a, bn)) continue;
      if (s2 && !conv_resident_s2_ok(rec.dt, rec.a, bn)) continue;
      for (int tw : widths) {
        if (halo && tw != 16) continue;  // the halo kernels' block is 16 x 16
        const int th = 256 / tw;
        const long area = (long)((rec.a.Ho + th - 1) / th) * th * ((rec.a.Wo + tw - 1) / tw) * tw;
        if (!halo && area * 10 > min_area * 11) continue;  // within 10 % of the least padding
        ConvArgs a = rec.a;
        a.tile_w = tw;
        if (halo_big && !conv_halo_tile_ok(rec.dt, a)) continue;
        a.amax = nullptr;
        res = check(launch_conv(rec.dt, tiles[ti], a, stream_), "autotune warm-up");
        if (!res.good()) break;
        res = check(hipEventRecord(e0, stream_), "hipEventRecord");
        const int reps = 2;
        for (int k = 0; res.good() && k < reps; ++k)
          res = check(launch_conv(rec.dt, tiles[ti], a, stream_), "autotune launch");
        if (res.good()) res = check(hipEventRecord(e1, stream_), "hipEventRecord");
        if (res.good()) res = check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        if (res.good()) res = check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (!res.good()) break;
        ms /= reps;
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          best = TuneVal{tiles[ti], tw};
        }
      }
    }
    if (res.good() && best_ms >= 0.f) found[rec.key] = best;
  }
  hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  recs_.clear();
  FFV_TRY(res);
  for (auto& kv : found) tuned_[kv.first] = kv.second;
  FFV_TRY(check(hipStreamSynchronize(stream_), "hipStreamSynchronize"));
  drop_graphs();  // captured with the previous tile choices
  if (n_tuned) *n_tuned = (int)found.size();
  return Status::ok();
}

static std::string tile_name(ConvTile t) {
  const std::string n = std::to_string(conv_tile_bn(t));
  if (t == ConvTile::R32 || t == ConvTile::R64) return "r" + n;
  if (t == ConvTile::S32 || t == ConvTile::S64 || t == ConvTile::S128) return "s" + n;
  if (t == ConvTile::Q256) return "q256";
  if (t == ConvTile::P256) return "p256";
  return (t == ConvTile::H32 || t == ConvTile::H256 || t == ConvTile::H128) ? "h" + n : n;
}

Status Net::save_tuning(const std::string& path) {
  std::lock_guard<std::mutex> lk(call_mu_);
  FILE* f = std::fopen(path.c_str(), "w");
  if (!f) return Status::err(-1, "cannot open " + path + " for writing");
  std::fprintf(f, "# ffv conv tuning v1: layer fp8 Ho Wo n_img n_tile tile_w\n");
  for (auto& kv : tuned_)
    std::fprintf(f, "%s %d %d %d %d %s %d\n", kv.first.layer.c_str(), kv.first.fp8, kv.first.Ho,
                 kv.first.Wo, kv.first.n_img, tile_name(kv.second.tile).c_str(), kv.second.tile_w);
  const bool ok = std::fclose(f) == 0;
  return ok ? Status::ok() : Status::err(-1, "write failed: " + path);
}

Status Net::load_tuning(const std::string& path, int* n_loaded) {
  ServingPause pause(sched_.get());
  std::lock_guard<std::mutex> lk(call_mu_);
  if (n_loaded) *n_loaded = 0;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return Status::err(-1, "cannot open " + path);
  std::map<TuneKey, TuneVal> got;
  char line[512];
  int lineno = 0;
  Status st = Status::ok();
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    char name[256], tname[16];
    int fp8, ho, wo, n, tw;
    if (std::sscanf(line, "%255s %d %d %d %d %15s %d", name, &fp8, &ho, &wo, &n, tname, &tw) != 7 ||
        (fp8 != 0 && fp8 != 1) || ho <= 0 || wo <= 0 || n <= 0 || tw <= 0 || tw > 256 || 256 % tw != 0 ||
        !layers_.count(name)) {
      st = Status::err(-1, path + ": bad entry on line " + std::to_string(lineno));
      break;
    }
    const std::string tn = tname;
    ConvTile t;
    if (tn == "256") t = ConvTile::N256;
    else if (tn == "128") t = ConvTile::N128;
    else if (tn == "64") t = ConvTile::N64;
    else if (tn == "32") t = ConvTile::N32;
    else if (tn == "h32" && tw == 16) t = ConvTile::H32;
    else if (tn == "h256" && (tw == 8 || tw == 16 || tw == 32)) t = ConvTile::H256;
    else if (tn == "h128" && (tw == 8 || tw == 16 || tw == 32)) t = ConvTile::H128;
    else if (tn == "q256" && (tw == 8 || tw == 16 || tw == 32)) t = ConvTile::Q256;
    else if (tn == "p256" && (tw == 8 || tw == 16 || tw == 32)) t = ConvTile::P256;
    else if (tn == "r32" && tw == 16) t = ConvTile::R32;
    else if (tn == "r64" && tw == 16) t = ConvTile::R64;
    else if (tn == "s32" && tw == 16) t = ConvTile::S32;
    else if (tn == "s64" && tw == 16) t = ConvTile::S64;
    else if (tn == "s128" && tw == 16) t = ConvTile::S128;
    else {
      st = Status::err(-1, path + ": bad tile on line " + std::to_string(lineno));
      break;
    }
    const int bn = conv_tile_bn(t);
    const Layer& L = layers_.at(name);
    if (L.name == "unet.head" || bn > L.cout_pad) {
      st = Status::err(-1, path + ": entry on line " + std::to_string(lineno) + " does not fit its layer");
      break;
    }
    got[TuneKey{name, fp8, ho, wo, n}] = TuneVal{t, tw};
  }
  std::fclose(f);
  FFV_TRY(st);
  for (auto& kv : got) tuned_[kv.first] = kv.second;
  if (stream_) hipStreamSynchronize(stream_);
  drop_graphs();
  if (n_loaded) *n_loaded = (int)got.size();
  return Status::ok();
}

Status Net::start_serving(size_t budget, float tick_ms, int max_batch_views) {
  if (sched_) return Status::err(kErrState, "serving already started");
  exec_.reset(new HipExecutor(this));
  Status st = exec_->init();
  if (st.good()) {
    sched_.reset(new Scheduler(exec_.get(), budget, tick_ms, max_batch_views));
    st = sched_->start();
  }
  if (!st.good()) {
    sched_.reset();
    exec_.reset();
  }
  return st;
}

}  // namespace ffv
