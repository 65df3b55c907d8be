// Serving scheduler (see scheduler.h). The completion callback takes no lock
// (atomics only): the scheduler may wait on the device while holding its
// lock, and a callback that waited for that lock could block the stream the
// device waits on.
#include "scheduler.h"

#include <algorithm>

#include <chrono>

namespace ffv {

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Scheduler::Scheduler(Executor* ex, size_t budget, float tick_ms, int max_batch)
    : ex_(ex),
      budget_(budget),
      tick_ms_(tick_ms > 0 ? tick_ms : 5.f),
      max_batch_(max_batch > 0 ? max_batch : 64) {}

Scheduler::~Scheduler() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (thr_.joinable()) thr_.join();
  for (auto& s : slots_)
    if (s->h) ex_->slot_wait(s->h);
  // callbacks may still be returning: wait until every slot reads free
  for (;;) {
    bool busy = false;
    for (auto& s : slots_) busy = busy || s->busy.load(std::memory_order_acquire);
    if (!busy) break;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  for (auto& s : slots_)
    if (s->h) ex_->slot_destroy(s->h);
  for (auto& kv : cams_)
    if (kv.second.handle) ex_->camera_destroy(kv.second.handle);
}

Status Scheduler::start() {
  for (int i = kMaxCams - 1; i >= 0; --i) free_cam_index_.push_back(i);
  thr_ = std::thread([this] { loop(); });
  return Status::ok();
}

bool Scheduler::any_busy() const {
  for (auto& s : slots_)
    if (s->busy.load(std::memory_order_acquire)) return true;
  return false;
}

bool Scheduler::camera_size(int id, int* H, int* W) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = cams_.find(id);
  if (it == cams_.end()) return false;
  *H = it->second.H;
  *W = it->second.W;
  return true;
}

void Scheduler::pause() {
  std::unique_lock<std::mutex> lk(mu_);
  ++paused_;
  while (any_busy()) cv_.wait_for(lk, std::chrono::milliseconds(1));
}

void Scheduler::resume() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    --paused_;
  }
  cv_.notify_all();
}

Status Scheduler::register_camera(int id, const float* image, int H, int W) {
  if (!image || H < 2 || W < 2) return Status::err(kErrArg, "bad camera image");
  std::unique_lock<std::mutex> lk(mu_);
  while (paused_ > 0) cv_.wait(lk);
  const size_t bytes = ex_->camera_bytes(H, W);
  size_t old_bytes = 0;
  auto it = cams_.find(id);
  if (it != cams_.end()) {
    // Queued tickets of this camera were sized for it: a replacement must
    // keep the size.
    if (it->second.H != H || it->second.W != W)
      return Status::err(kErrArg, "a registered camera can only be replaced by an image of the same size");
    // wait until no batch in flight can reference the camera
    while (any_busy()) cv_.wait_for(lk, std::chrono::milliseconds(1));
    old_bytes = ex_->camera_bytes(it->second.H, it->second.W);
  } else if (free_cam_index_.empty()) {
    return Status::err(kErrArg, "too many cameras");
  }
  if (resident_bytes_ - old_bytes + bytes + slot_bytes_ > budget_)
    return Status::err(kErrBudget, "camera does not fit the HBM budget");
  const int index = it != cams_.end() ? it->second.index : free_cam_index_.back();
  void* h = nullptr;
  if (it != cams_.end()) {
    // the old data goes first, so both never need to fit at once
    ex_->camera_destroy(it->second.handle);
    it->second.handle = nullptr;
    resident_bytes_ -= old_bytes;
  }
  Status st = ex_->camera_create(index, image, H, W, &h);
  if (!st.good()) {
    if (it != cams_.end()) {
      // the id stays known but has no data: requests for it fail at submit
      free_cam_index_.push_back(index);
      cams_.erase(it);
    }
    return st;
  }
  if (it == cams_.end()) free_cam_index_.pop_back();
  Camera c;
  c.H = H;
  c.W = W;
  c.handle = h;
  c.index = index;
  cams_[id] = c;
  resident_bytes_ += bytes;
  return Status::ok();
}

Status Scheduler::check_locked(const Request& r, int* H, int* W) const {
  if (!r.out) return Status::err(kErrArg, "null output pointer");
  if (!(r.t >= 0.f && r.t <= 1.f)) return Status::err(kErrArg, "t must lie in [0, 1]");
  auto a = cams_.find(r.cam_l), b = cams_.find(r.cam_r);
  if (a == cams_.end() || b == cams_.end()) return Status::err(kErrArg, "unknown camera id");
  if (a->second.H != b->second.H || a->second.W != b->second.W)
    return Status::err(kErrArg, "cameras of a pair differ in size");
  *H = a->second.H;
  *W = a->second.W;
  if (resident_bytes_ + ex_->batch_bytes(*H, *W, 1) > budget_)
    return Status::err(kErrBudget, "request can never fit the HBM budget");
  return Status::ok();
}

uint64_t Scheduler::enqueue_locked(const Request& r, int H, int W) {
  const uint64_t id = next_ticket_++;
  Ticket& t = tickets_[id];
  t.req = r;
  t.H = H;
  t.W = W;
  t.tm.t_submit = now_seconds();
  t.state.store(0, std::memory_order_relaxed);
  queue_.push_back(id);
  return id;
}

Status Scheduler::submit(const Request& r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(mu_);
  int H = 0, W = 0;
  const Status st = check_locked(r, &H, &W);
  if (!st.good()) return st;
  // admitted at the next tick or when a running batch completes
  *ticket = enqueue_locked(r, H, W);
  return Status::ok();
}

Status Scheduler::submit_many(const Request* rs, int n, uint64_t* tickets, int* bad) {
  if (bad) *bad = -1;
  if (n < 0 || (n > 0 && (!rs || !tickets))) return Status::err(kErrArg, "bad request array");
  std::lock_guard<std::mutex> lk(mu_);
  std::vector<std::pair<int, int>> hw(n);
  for (int i = 0; i < n; ++i) {
    const Status st = check_locked(rs[i], &hw[i].first, &hw[i].second);
    if (!st.good()) {
      if (bad) *bad = i;
      return st;
    }
  }
  for (int i = 0; i < n; ++i) tickets[i] = enqueue_locked(rs[i], hw[i].first, hw[i].second);
  return Status::ok();
}

Status Scheduler::poll(uint64_t ticket, Timing* timing, bool* done) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(ticket);
  if (it == tickets_.end()) return Status::err(kErrTicket, "unknown or collected ticket");
  const int state = it->second.state.load(std::memory_order_acquire);
  if (state == 3) {
    const Status st = it->second.err;
    tickets_.erase(it);
    *done = true;
    return st;
  }
  if (state != 2) {
    *done = false;
    return Status::ok();
  }
  if (timing) *timing = it->second.tm;
  tickets_.erase(it);
  *done = true;
  return Status::ok();
}

Status Scheduler::stats(long* admitted, long* completed, long* queued, size_t* bytes_in_use) {
  std::lock_guard<std::mutex> lk(mu_);
  *admitted = n_admitted_;
  *completed = n_completed_.load();
  *queued = (long)queue_.size();
  *bytes_in_use = resident_bytes_ + slot_bytes_;
  return Status::ok();
}

void Scheduler::on_done(void* p) {
  Done* d = static_cast<Done*>(p);
  Scheduler* s = d->s;
  Slot& sl = *d->slot;
  const double t = now_seconds();
  for (Ticket* tk : sl.tickets) {
    tk->tm.t_done = t;
    tk->state.store(2, std::memory_order_release);
  }
  s->n_completed_.fetch_add((long)sl.tickets.size());
  s->cv_.notify_all();
  // last: once the slot reads free, the scheduler may be destroyed
  sl.busy.store(false, std::memory_order_release);
}

void Scheduler::fail_tickets(const std::vector<Ticket*>& tks, const Status& st) {
  const double t = now_seconds();
  for (Ticket* tk : tks) {
    tk->err = st;
    tk->tm.t_done = t;
    tk->state.store(3, std::memory_order_release);
  }
}

void Scheduler::admit_and_launch() {
  while (!queue_.empty() && paused_ == 0) {
    // FIFO over the queue, at most kMaxSizes resolutions in a batch
    std::vector<size_t> pick;
    std::vector<std::pair<int, int>> sizes;
    for (size_t i = 0; i < queue_.size() && (int)pick.size() < max_batch_; ++i) {
      const Ticket& t = tickets_[queue_[i]];
      const std::pair<int, int> hw(t.H, t.W);
      if (std::find(sizes.begin(), sizes.end(), hw) == sizes.end()) {
        if ((int)sizes.size() == kMaxSizes) continue;
        sizes.push_back(hw);
      }
      pick.push_back(i);
    }
    int n = (int)pick.size();
    // the largest height and width among the first m picks
    auto max_size = [&](int m, int* H, int* W) {
      *H = *W = 0;
      for (int i = 0; i < m; ++i) {
        const Ticket& t = tickets_[queue_[pick[i]]];
        *H = std::max(*H, t.H);
        *W = std::max(*W, t.W);
      }
    };
    int H = 0, W = 0;
    // a free slot large enough, or room in the budget for one
    Slot* slot = nullptr;
    int slot_idx = -1;
    Status alloc_err;
    while (n >= 1 && !slot) {
      max_size(n, &H, &W);
      const size_t need = ex_->batch_bytes(H, W, n);
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
          if (resident_bytes_ + slot_bytes_ - s.bytes + need > budget_) continue;
          slot_bytes_ -= s.bytes;
          s.bytes = 0;
          Status st = ex_->slot_resize(s.h, need);
          if (st.good()) {
            s.bytes = need;
            slot_bytes_ += need;
            slot = &s;
            slot_idx = (int)i;
          } else {
            alloc_err = st;
          }
        }
        if (!slot && resident_bytes_ + slot_bytes_ + need <= budget_) {
          void* h = nullptr;
          Status st = ex_->slot_create(need, &h);
          if (st.good()) {
            std::unique_ptr<Slot> s(new Slot());
            s->h = h;
            s->bytes = need;
            slot_bytes_ += need;
            slots_.push_back(std::move(s));
            done_ctx_.emplace_back(new Done{this, slots_.back().get()});
            slot = slots_.back().get();
            slot_idx = (int)slots_.size() - 1;
          } else {
            alloc_err = st;
          }
        }
      }
      if (!slot) n /= 2;
    }
    if (!slot) {
      // Nothing in flight will free memory: the head request cannot run now.
      if (!alloc_err.good() && !any_busy()) {
        Ticket& t = tickets_[queue_.front()];
        queue_.pop_front();
        fail_tickets({&t}, alloc_err);
        continue;
      }
      return;  // wait for a slot to free up
    }

    pick.resize(n);
    const double t_admit = now_seconds();
    std::vector<ViewJob> jobs(n);
    std::vector<Ticket*> tks(n);
    for (int i = 0; i < n; ++i) {
      const uint64_t id = queue_[pick[i]];
      Ticket& t = tickets_[id];
      t.state.store(1, std::memory_order_relaxed);
      t.tm.t_admit = t_admit;
      tks[i] = &t;
      ViewJob& j = jobs[i];
      j.cam_l = cams_[t.req.cam_l].index;
      j.cam_r = cams_[t.req.cam_r].index;
      j.t = t.req.t;
      j.out = t.req.out;
      j.H = t.H;
      j.W = t.W;
    }
    for (int i = n - 1; i >= 0; --i) queue_.erase(queue_.begin() + pick[i]);
    slot->tickets = tks;
    slot->busy.store(true, std::memory_order_release);
    n_admitted_ += n;
    const Status st = ex_->launch(slot->h, H, W, jobs.data(), n, &Scheduler::on_done,
                                  done_ctx_[slot_idx].get());
    if (!st.good()) {
      // nothing of the batch is running: its tickets fail with the status
      fail_tickets(tks, st);
      slot->tickets.clear();
      slot->busy.store(false, std::memory_order_release);
      continue;
    }
    // t_launch is not touched by the callback; poll reads it under the lock
    const double t_launch = now_seconds();
    for (Ticket* tk : tks) tk->tm.t_launch = t_launch;
  }
}

void Scheduler::loop() {
  std::unique_lock<std::mutex> lk(mu_);
  while (!stop_) {
    admit_and_launch();
    cv_.wait_for(lk, std::chrono::microseconds((long)(tick_ms_ * 1000)));
  }
}

}  // namespace ffv
