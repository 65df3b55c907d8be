// Serving scheduler: continuous batching of viewpoint requests over
// resident cameras under an HBM admission budget.
//
// Every tick (or when a request arrives) the scheduler admits queued
// requests in FIFO order, grouping those of one resolution into a batch of
// at most max_batch views, if a slot (a stream with its own workspace) is
// free or can be created within the budget. A batch runs on its slot's
// stream, so batches of consecutive ticks overlap on the device; a host
// callback queued behind the batch marks its tickets done and frees the
// slot. The callback takes no lock (atomics only): the scheduler may make
// device-synchronising calls while holding its lock, and a callback that
// waited for that lock would block the stream the device waits on. The
// per-view arithmetic does not depend on the batch a view lands in, so a
// request's result is the same alone or in any mix.
#include <algorithm>
#include <chrono>

#include "net.h"

namespace ffv {

Server::Server(Net* net, size_t budget, float tick_ms, int max_batch_views)
    : net_(net),
      budget_(budget),
      tick_ms_(tick_ms > 0 ? tick_ms : 5.f),
      max_batch_(max_batch_views > 0 ? max_batch_views : 64) {}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (thr_.joinable()) thr_.join();
  hipSetDevice(net_->device());
  for (auto& s : slots_)
    if (s->s) hipStreamSynchronize(s->s);
  for (auto& s : slots_) {
    if (s->ws) hipFree(s->ws);
    if (s->s) hipStreamDestroy(s->s);
  }
  for (auto& kv : cams_)
    if (kv.second.block) hipFree(kv.second.block);
  if (cam_table_) hipFree(cam_table_);
}

Status Server::start() {
  Status st = net_->check(hipSetDevice(net_->device()), "hipSetDevice");
  if (!st.good()) return st;
  st = net_->check(hipMalloc((void**)&cam_table_, sizeof(CamDev) * kMaxCams), "hipMalloc camera table");
  if (!st.good()) return st;
  for (int i = kMaxCams - 1; i >= 0; --i) free_cam_slots_.push_back(i);
  thr_ = std::thread([this] { loop(); });
  return Status::ok();
}

size_t Server::view_bytes(const Geo& g, int n) const { return net_->view_plan(g, n).total; }

Status Server::register_camera(int cam_id, const float* image, int H, int W) {
  if (!image || H < 2 || W < 2) return Status::err(-1, "bad camera image");
  std::unique_lock<std::mutex> lk(mu_);
  hipSetDevice(net_->device());
  const Geo g = Geo::of(H, W);
  const CamPlan cp = net_->cam_plan(g);
  size_t old_bytes = 0;
  auto it = cams_.find(cam_id);
  if (it != cams_.end()) {
    // replacing: wait until no batch in flight can reference the camera
    for (;;) {
      bool any = false;
      for (auto& s : slots_) any = any || s->busy.load(std::memory_order_acquire);
      if (!any) break;
      cv_.wait_for(lk, std::chrono::milliseconds(1));
    }
    old_bytes = net_->cam_plan(it->second.g).bytes;
  } else if (free_cam_slots_.empty()) {
    return Status::err(-1, "too many cameras");
  }
  if (resident_bytes_ - old_bytes + cp.bytes + slot_bytes_ > budget_)
    return Status::err(-3, "camera does not fit the HBM budget");

  char* block = nullptr;
  char* tmp = nullptr;
  hipStream_t s = nullptr;
  auto cleanup = [&]() {
    if (tmp) hipFree(tmp);
    if (s) hipStreamDestroy(s);
  };
  Status st = net_->check(hipMalloc((void**)&block, cp.bytes), "hipMalloc camera");
  if (st.good())
    st = net_->check(hipMalloc((void**)&tmp, cp.ctmp + 256), "hipMalloc scratch");
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
  }
  if (!st.good()) {
    if (block) hipFree(block);
    cleanup();
    return st;
  }
  cleanup();
  Camera c;
  c.g = g;
  c.block = block;
  if (it != cams_.end()) {
    c.slot = it->second.slot;
    hipFree(it->second.block);
    resident_bytes_ -= old_bytes;
  } else {
    c.slot = free_cam_slots_.back();
    free_cam_slots_.pop_back();
  }
  const CamDev d = net_->cam_dev(g, block);
  st = net_->check(hipMemcpy(cam_table_ + c.slot, &d, sizeof(CamDev), hipMemcpyHostToDevice),
                   "copy camera entry");
  if (!st.good()) return st;
  cams_[cam_id] = c;
  resident_bytes_ += cp.bytes;
  return Status::ok();
}

Status Server::submit(const Request& r, uint64_t* ticket) {
  if (!r.out) return Status::err(-1, "null output pointer");
  if (!net_->ready()) return Status::err(-7, "FP8 net needs ffv_calibrate first");
  if (!(r.t >= 0.f && r.t <= 1.f)) return Status::err(-1, "t must lie in [0, 1]");
  std::lock_guard<std::mutex> lk(mu_);
  auto a = cams_.find(r.cam_l), b = cams_.find(r.cam_r);
  if (a == cams_.end() || b == cams_.end()) return Status::err(-1, "unknown camera id");
  if (!(a->second.g == b->second.g)) return Status::err(-1, "cameras of a pair differ in size");
  const Geo g = a->second.g;
  if (resident_bytes_ + view_bytes(g, 1) > budget_)
    return Status::err(-3, "request can never fit the HBM budget");
  const uint64_t id = next_ticket_++;
  Ticket& t = tickets_[id];
  t.req = r;
  t.g = g;
  t.tm.t_submit = now_seconds();
  t.state.store(0, std::memory_order_relaxed);
  queue_.push_back(id);
  *ticket = id;
  // admitted at the next tick or when a running batch completes
  return Status::ok();
}

Status Server::poll(uint64_t ticket, Timing* timing, bool* done) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return Status::err(-6, "unknown or collected ticket");
  if (it->second.state.load(std::memory_order_acquire) != 2) {
    *done = false;
    return Status::ok();
  }
  if (timing) *timing = it->second.tm;
  tickets_.erase(it);
  *done = true;
  return Status::ok();
}

Status Server::stats(long* admitted, long* completed, long* queued, size_t* bytes_in_use) {
  std::lock_guard<std::mutex> lk(mu_);
  *admitted = n_admitted_;
  *completed = n_completed_.load();
  *queued = (long)queue_.size();
  *bytes_in_use = resident_bytes_ + slot_bytes_;
  return Status::ok();
}

void Server::on_done(void* p) {
  Done* d = static_cast<Done*>(p);
  Server* s = d->srv;
  Slot& sl = *d->slot;
  const double t = now_seconds();
  for (Ticket* tk : sl.tickets) {
    tk->tm.t_done = t;
    tk->state.store(2, std::memory_order_release);
  }
  s->n_completed_.fetch_add((long)sl.tickets.size());
  sl.busy.store(false, std::memory_order_release);
  s->cv_.notify_all();
}

void Server::admit_and_launch() {
  while (!queue_.empty()) {
    const Geo g = tickets_[queue_.front()].g;
    // FIFO within one resolution
    std::vector<size_t> pick;
    for (size_t i = 0; i < queue_.size() && (int)pick.size() < max_batch_; ++i)
      if (tickets_[queue_[i]].g == g) pick.push_back(i);
    int n = (int)pick.size();
    // a free slot large enough, or room in the budget for one
    Slot* slot = nullptr;
    int slot_idx = -1;
    while (n >= 1 && !slot) {
      const size_t need = view_bytes(g, n);
      for (size_t i = 0; i < slots_.size(); ++i)
        if (!slots_[i]->busy.load(std::memory_order_acquire) && slots_[i]->bytes >= need) {
          slot = slots_[i].get();
          slot_idx = (int)i;
          break;
        }
      if (!slot) {
        // grow a free slot, or add one, within the budget
        for (size_t i = 0; i < slots_.size() && !slot; ++i) {
          Slot& s = *slots_[i];
          if (s.busy.load(std::memory_order_acquire)) continue;
          if (resident_bytes_ + slot_bytes_ - s.bytes + need <= budget_) {
            hipFree(s.ws);
            slot_bytes_ -= s.bytes;
            s.ws = nullptr;
            s.bytes = 0;
            if (hipMalloc((void**)&s.ws, need) == hipSuccess) {
              s.bytes = need;
              slot_bytes_ += need;
              slot = &s;
              slot_idx = (int)i;
            }
          }
        }
        if (!slot && resident_bytes_ + slot_bytes_ + need <= budget_) {
          std::unique_ptr<Slot> s(new Slot());
          if (hipStreamCreateWithFlags(&s->s, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void**)&s->ws, need) == hipSuccess) {
            s->bytes = need;
            slot_bytes_ += need;
            slots_.push_back(std::move(s));
            done_ctx_.emplace_back(new Done{this, slots_.back().get()});
            slot = slots_.back().get();
            slot_idx = (int)slots_.size() - 1;
          } else {
            if (s->ws) hipFree(s->ws);
            if (s->s) hipStreamDestroy(s->s);
          }
        }
      }
      if (!slot) n /= 2;
    }
    if (!slot) return;  // wait for a slot to free up

    pick.resize(n);
    const double t_admit = now_seconds();
    std::vector<ViewDesc> vd(n);
    std::vector<Ticket*> tks(n);
    for (int i = 0; i < n; ++i) {
      const uint64_t id = queue_[pick[i]];
      Ticket& t = tickets_[id];
      t.state.store(1, std::memory_order_relaxed);
      t.tm.t_admit = t_admit;
      tks[i] = &t;
      ViewDesc& d = vd[i];
      d = ViewDesc{};
      d.cam_l = cams_[t.req.cam_l].slot;
      d.cam_r = cams_[t.req.cam_r].slot;
      d.t = t.req.t;
      d.out = t.req.out;
    }
    for (int i = n - 1; i >= 0; --i) queue_.erase(queue_.begin() + pick[i]);
    slot->busy.store(true, std::memory_order_relaxed);
    slot->tickets = tks;
    n_admitted_ += n;
    Exec x;
    x.s = slot->s;
    x.ws = slot->ws;
    const ViewPlan vp = net_->view_plan(g, n);
    Status st = net_->run_views(x, vp, cam_table_, vd.data(), n);
    const double t_launch = now_seconds();
    for (Ticket* tk : tks) tk->tm.t_launch = t_launch;
    if (!st.good() ||
        hipLaunchHostFunc(slot->s, &Server::on_done, done_ctx_[slot_idx].get()) != hipSuccess) {
      // the batch could not be queued: wait for what was, report it done
      // (outputs undefined)
      hipStreamSynchronize(slot->s);
      on_done(done_ctx_[slot_idx].get());
      return;
    }
  }
}

void Server::loop() {
  hipSetDevice(net_->device());
  std::unique_lock<std::mutex> lk(mu_);
  while (!stop_) {
    admit_and_launch();
    cv_.wait_for(lk, std::chrono::microseconds((long)(tick_ms_ * 1000)));
  }
}

}  // namespace ffv
