// Device side of the serving scheduler (scheduler.h): resident camera data,
// batch workspaces on their own streams, and the network's launches for a
// batch of views, completed by a host function queued behind them.
#include "serve.h"

#include <algorithm>
#include <map>
#include <numeric>
#include <vector>

#include "fault.h"

namespace ffv {

namespace {

// A slot's captured batches: one graph per batch layout (the size groups'
// heights, widths and view counts), valid for the slot's current workspace
// and the net's graph epoch.
struct HSlot {
  hipStream_t s = nullptr;
  char* ws = nullptr;
  size_t bytes = 0;
  uint64_t epoch = 0;
  std::map<std::vector<int>, hipGraphExec_t> graphs;
  void drop_graphs() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
};

}  // namespace

HipExecutor::~HipExecutor() {
  if (cam_table_) hipFree(cam_table_);
}

Status HipExecutor::init() {
  Status st = net_->check(hipSetDevice(net_->device()), "hipSetDevice");
  if (!st.good()) return st;
  return net_->dev_alloc((void**)&cam_table_, sizeof(CamDev) * Scheduler::kMaxCams, "camera table");
}

size_t HipExecutor::camera_bytes(int H, int W) const { return net_->cam_plan(Geo::of(H, W)).bytes; }

size_t HipExecutor::batch_bytes(int H, int W, int n) const {
  return net_->view_plan(Geo::of(H, W), n).total;
}

Status HipExecutor::camera_create(int index, const float* image, int H, int W, void** cam) {
  if (index < 0 || index >= Scheduler::kMaxCams) return Status::err(kErrArg, "camera index");
  hipSetDevice(net_->device());
  const Geo g = Geo::of(H, W);
  const CamPlan cp = net_->cam_plan(g);
  char* block = nullptr;
  char* tmp = nullptr;
  hipStream_t s = nullptr;
  Status st = net_->dev_alloc((void**)&block, cp.bytes, "camera");
  if (st.good()) st = net_->dev_alloc((void**)&tmp, cp.ctmp + 256, "camera scratch");
  if (st.good()) st = net_->check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
  if (st.good()) {
    const float** src_tab = (const float**)(tmp + cp.ctmp);
    st = net_->check(hipMemcpyAsync(src_tab, &image, sizeof(void*), hipMemcpyHostToDevice, s),
                     "copy image pointer");
    if (st.good()) {
      Exec x;
      x.s = s;
      char* blocks[1] = {block};
      st = net_->build_cameras(x, g, src_tab, 1, blocks, tmp);
    }
    if (st.good()) st = net_->check(hipStreamSynchronize(s), "sync camera build");
    else hipStreamSynchronize(s);
  }
  if (st.good()) {
    // no batch in flight reads this entry: a new index is unused, and a
    // replaced camera is rebuilt only once the slots are idle
    const CamDev d = net_->cam_dev(g, block);
    st = net_->check(hipMemcpy(cam_table_ + index, &d, sizeof(CamDev), hipMemcpyHostToDevice),
                     "copy camera entry");
  }
  if (tmp) hipFree(tmp);
  if (s) hipStreamDestroy(s);
  if (!st.good()) {
    if (block) hipFree(block);
    return st;
  }
  *cam = block;
  return Status::ok();
}

void HipExecutor::camera_destroy(void* cam) {
  hipSetDevice(net_->device());
  hipFree(cam);
}

Status HipExecutor::slot_create(size_t bytes, void** slot) {
  hipSetDevice(net_->device());
  HSlot* h = new HSlot();
  Status st = net_->check(hipStreamCreateWithFlags(&h->s, hipStreamNonBlocking), "slot stream");
  if (st.good()) st = net_->dev_alloc((void**)&h->ws, bytes, "slot workspace");
  if (!st.good()) {
    if (h->s) hipStreamDestroy(h->s);
    delete h;
    return st;
  }
  h->bytes = bytes;
  *slot = h;
  return Status::ok();
}

Status HipExecutor::slot_resize(void* slot, size_t bytes) {
  HSlot* h = static_cast<HSlot*>(slot);
  hipSetDevice(net_->device());
  h->drop_graphs();  // they address the old workspace
  if (h->ws) hipFree(h->ws);
  h->ws = nullptr;
  h->bytes = 0;
  Status st = net_->dev_alloc((void**)&h->ws, bytes, "slot workspace");
  if (st.good()) h->bytes = bytes;
  return st;
}

void HipExecutor::slot_destroy(void* slot) {
  HSlot* h = static_cast<HSlot*>(slot);
  hipSetDevice(net_->device());
  if (h->s) hipStreamSynchronize(h->s);
  h->drop_graphs();
  if (h->ws) hipFree(h->ws);
  if (h->s) hipStreamDestroy(h->s);
  delete h;
}

void HipExecutor::slot_wait(void* slot) {
  HSlot* h = static_cast<HSlot*>(slot);
  if (h->s) hipStreamSynchronize(h->s);
}

Status HipExecutor::launch(void* slot, int H, int W, const ViewJob* jobs, int n, void (*done)(void*),
                           void* ctx) {
  HSlot* h = static_cast<HSlot*>(slot);
  if (fault_hit("launch")) return Status::err(kErrDevice, "injected launch fault (FFV_FAULT)");
  hipSetDevice(net_->device());
  // views ordered by size (stable), one group per size; the workspace is
  // planned for the largest height and width
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return jobs[a].H != jobs[b].H ? jobs[a].H < jobs[b].H : jobs[a].W < jobs[b].W;
  });
  std::vector<ViewGroup> groups;
  std::vector<int> key;
  for (int i = 0; i < n; ++i) {
    const ViewJob& j = jobs[order[i]];
    if (j.H < 2 || j.W < 2 || j.H > H || j.W > W) return Status::err(kErrArg, "view size");
    const Geo gj = Geo::of(j.H, j.W);
    if (groups.empty() || groups.back().Hp != gj.Hp || groups.back().Wp != gj.Wp ||
        jobs[order[i - 1]].H != j.H || jobs[order[i - 1]].W != j.W) {
      if ((int)groups.size() == ConvGroup::kMax) return Status::err(kErrArg, "too many view sizes in a batch");
      groups.push_back(ViewGroup{i, 0, gj.Hp, gj.Wp});
      key.insert(key.end(), {j.H, j.W, 0});
    }
    ++groups.back().n;
    ++key.back();
  }
  const Geo g = Geo::of(H, W);
  const ViewPlan vp = net_->view_plan(g, n);
  if (vp.total > h->bytes) return Status::err(kErrArg, "batch larger than its slot");
  std::vector<ViewDesc> vd(n);
  for (int i = 0; i < n; ++i) {
    const ViewJob& j = jobs[order[i]];
    const Geo gj = Geo::of(j.H, j.W);
    vd[i] = ViewDesc{};
    vd[i].cam_l = j.cam_l;
    vd[i].cam_r = j.cam_r;
    vd[i].t = j.t;
    vd[i].out = j.out;
    vd[i].hp = gj.Hp;
    vd[i].wp = gj.Wp;
    vd[i].h = gj.H;
    vd[i].w = gj.W;
  }
  Exec x;
  x.s = h->s;
  x.ws = h->ws;
  if (groups.size() > 1) {
    x.groups = groups.data();
    x.n_groups = (int)groups.size();
    x.plan_hp = g.Hp;
  }
  key.insert(key.begin(), {H, W});
  Status st;
  if (net_->graphs_enabled()) {
    // The batch's view descriptors go to the slot's device table first, so a
    // captured graph holds no per-request value and replays for any batch of
    // the same shape on this slot.
    ViewDesc* tab = (ViewDesc*)x.at(vp.views);
    st = net_->check(hipMemcpyAsync(tab, vd.data(), sizeof(ViewDesc) * n, hipMemcpyHostToDevice, h->s),
                     "copy views");
    const uint64_t epoch = net_->graph_epoch();
    if (h->epoch != epoch) {
      h->drop_graphs();
      h->epoch = epoch;
    }
    auto it = h->graphs.find(key);
    if (st.good() && it == h->graphs.end()) {
      if (h->graphs.size() >= 128) h->drop_graphs();  // bound the cache (batch shapes vary)
      st = net_->check(hipStreamBeginCapture(h->s, hipStreamCaptureModeThreadLocal), "begin capture");
      if (st.good()) {
        x.capture = true;
        Status run = net_->run_views(x, vp, cam_table_, tab, n, true);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->s, &graph);
        hipGraphExec_t exec = nullptr;
        if (run.good() && ec == hipSuccess) run = net_->check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0),
                                                             "graph instantiate");
        else if (run.good()) run = net_->check(ec, "end capture");
        if (graph) hipGraphDestroy(graph);
        st = run;
        if (st.good()) it = h->graphs.emplace(key, exec).first;
      }
    }
    if (st.good()) st = net_->check(hipGraphLaunch(it->second, h->s), "graph launch");
  } else {
    st = net_->run_views(x, vp, cam_table_, vd.data(), n);
  }
  if (st.good()) st = net_->check(hipLaunchHostFunc(h->s, done, ctx), "hipLaunchHostFunc");
  if (!st.good()) {
    // part of the batch may be queued: let it finish before the slot is reused
    hipStreamSynchronize(h->s);
    return st;
  }
  return Status::ok();
}

}  // namespace ffv
