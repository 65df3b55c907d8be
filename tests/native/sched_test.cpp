// Host-only tests of the serving scheduler (paper_2112_10603_amd/csrc/
// scheduler.cpp) behind a fake executor: no GPU, no HIP. Built with g++ by
// tests/test_sched_host.py, plainly and under AddressSanitizer +
// UndefinedBehaviorSanitizer and ThreadSanitizer.
//
// The fake executor stands in for the device: "device memory" is host
// memory whose live total is checked against the budget at every
// allocation, a slot is a worker thread that finishes a batch after a
// delay, and a batch "computes" each view by writing a value that depends
// only on that view's cameras and phase into its output buffer.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "fault.h"
#include "scheduler.h"

using namespace ffv;

static int g_failures = 0;
#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
      ++g_failures;                                                          \
    }                                                                        \
  } while (0)

// The value a view's output holds: depends on the view alone.
static float view_value(int cam_l, int cam_r, float t) { return cam_l * 1000.f + cam_r + t; }

struct Batch {
  int H, W;
  std::vector<ViewJob> jobs;
};

class FakeExecutor : public Executor {
 public:
  explicit FakeExecutor(size_t budget, int delay_ms) : budget_(budget), delay_ms_(delay_ms) {}
  ~FakeExecutor() override {}

  size_t camera_bytes(int H, int W) const override { return (size_t)H * W * 10; }
  size_t batch_bytes(int H, int W, int n) const override { return (size_t)n * H * W * 4; }

  Status camera_create(int index, const float* image, int H, int W, void** cam) override {
    if (!image) return Status::err(kErrArg, "image");
    void* p = nullptr;
    Status st = alloc(camera_bytes(H, W), &p);
    if (!st.good()) return st;
    std::lock_guard<std::mutex> lk(mu_);
    if (index < 0 || index >= Scheduler::kMaxCams) return Status::err(kErrArg, "index");
    cam_ids_[index] = (int)image[0];  // the test's "image" holds the camera id
    *cam = p;
    return Status::ok();
  }
  void camera_destroy(void* cam) override { release(cam); }

  struct Slot {
    std::mutex m;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    int inflight = 0;
    bool stop = false;
    std::thread th;
    void* ws = nullptr;
    size_t bytes = 0;
  };

  Status slot_create(size_t bytes, void** slot) override {
    Slot* s = new Slot();
    Status st = alloc(bytes, &s->ws);
    if (!st.good()) {
      delete s;
      return st;
    }
    s->bytes = bytes;
    s->th = std::thread([s] {
      std::unique_lock<std::mutex> lk(s->m);
      for (;;) {
        s->cv.wait(lk, [s] { return s->stop || !s->q.empty(); });
        if (s->q.empty()) return;
        auto f = std::move(s->q.front());
        s->q.pop_front();
        lk.unlock();
        f();
        lk.lock();
        --s->inflight;
        s->cv.notify_all();
      }
    });
    slots_created_.fetch_add(1);
    *slot = s;
    return Status::ok();
  }
  Status slot_resize(void* slot, size_t bytes) override {
    Slot* s = static_cast<Slot*>(slot);
    if (s->ws) release(s->ws);
    s->ws = nullptr;
    s->bytes = 0;
    Status st = alloc(bytes, &s->ws);
    if (st.good()) s->bytes = bytes;
    return st;
  }
  void slot_destroy(void* slot) override {
    Slot* s = static_cast<Slot*>(slot);
    {
      std::lock_guard<std::mutex> lk(s->m);
      s->stop = true;
    }
    s->cv.notify_all();
    s->th.join();
    if (s->ws) release(s->ws);
    delete s;
  }
  void slot_wait(void* slot) override {
    Slot* s = static_cast<Slot*>(slot);
    std::unique_lock<std::mutex> lk(s->m);
    s->cv.wait(lk, [s] { return s->inflight == 0; });
  }

  Status launch(void* slot, int H, int W, const ViewJob* jobs, int n, void (*done)(void*),
                void* ctx) override {
    if (fault_hit("launch")) return Status::err(kErrDevice, "injected launch fault");
    Slot* s = static_cast<Slot*>(slot);
    if (batch_bytes(H, W, n) > s->bytes) return Status::err(kErrArg, "batch larger than slot");
    for (int i = 0; i < n; ++i)
      if (jobs[i].H > H || jobs[i].W > W) return Status::err(kErrArg, "view larger than the batch");
    Batch b{H, W, std::vector<ViewJob>(jobs, jobs + n)};
    std::vector<int> ids(n * 2);
    {
      std::lock_guard<std::mutex> lk(mu_);
      batches_.push_back(b);
      for (int i = 0; i < n; ++i) {
        ids[2 * i] = cam_ids_[jobs[i].cam_l];
        ids[2 * i + 1] = cam_ids_[jobs[i].cam_r];
      }
      const int busy = ++busy_now_;
      if (busy > max_busy_) max_busy_ = busy;
    }
    const int delay = delay_ms_;
    std::lock_guard<std::mutex> lk(s->m);
    ++s->inflight;
    s->q.push_back([this, b, ids, delay, done, ctx] {
      std::this_thread::sleep_for(std::chrono::milliseconds(delay));
      for (size_t i = 0; i < b.jobs.size(); ++i)
        for (int k = 0; k < 3 * b.jobs[i].H * b.jobs[i].W; ++k)
          b.jobs[i].out[k] = view_value(ids[2 * i], ids[2 * i + 1], b.jobs[i].t);
      {
        std::lock_guard<std::mutex> g(mu_);
        --busy_now_;
      }
      done(ctx);
    });
    s->cv.notify_all();
    return Status::ok();
  }

  // test inspection
  std::vector<Batch> batches() {
    std::lock_guard<std::mutex> lk(mu_);
    return batches_;
  }
  size_t live_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return live_;
  }
  size_t peak_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return peak_;
  }
  int max_busy() {
    std::lock_guard<std::mutex> lk(mu_);
    return max_busy_;
  }
  int live_allocs() {
    std::lock_guard<std::mutex> lk(mu_);
    return (int)sizes_.size();
  }
  std::atomic<int> slots_created_{0};

 private:
  Status alloc(size_t bytes, void** p) {
    if (fault_hit("alloc")) return Status::err(kErrOom, "injected allocation fault");
    void* q = std::malloc(bytes ? bytes : 1);
    if (!q) return Status::err(kErrOom, "malloc");
    std::lock_guard<std::mutex> lk(mu_);
    sizes_.push_back({q, bytes});
    live_ += bytes;
    if (live_ > peak_) peak_ = live_;
    if (live_ > budget_) over_budget_ = true;
    *p = q;
    return Status::ok();
  }
  void release(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < sizes_.size(); ++i)
      if (sizes_[i].first == p) {
        live_ -= sizes_[i].second;
        sizes_.erase(sizes_.begin() + i);
        break;
      }
    std::free(p);
  }

 public:
  bool over_budget_ = false;

 private:
  size_t budget_;
  int delay_ms_;
  std::mutex mu_;
  std::vector<std::pair<void*, size_t>> sizes_;
  size_t live_ = 0, peak_ = 0;
  std::vector<Batch> batches_;
  int cam_ids_[Scheduler::kMaxCams] = {};
  int busy_now_ = 0, max_busy_ = 0;
};

// A camera "image": 3 x H x W floats whose first value is the camera id.
struct Image {
  std::vector<float> px;
  Image(int id, int H, int W) : px((size_t)3 * H * W, 0.f) { px[0] = (float)id; }
};

struct Out {
  std::vector<float> px;
  Out(int H, int W) : px((size_t)3 * H * W, -1.f) {}
  float* p() { return px.data(); }
};

// Poll until done (or a failure status); returns the status code.
static int wait_ticket(Scheduler& s, uint64_t tk, Timing* tm = nullptr, int timeout_ms = 5000) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    bool done = false;
    Timing t;
    Status st = s.poll(tk, &t, &done);
    if (!st.good()) return st.code;
    if (done) {
      if (tm) *tm = t;
      return 0;
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms)) return 99;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

static uint64_t submit(Scheduler& s, int l, int r, float t, float* out, int* code = nullptr) {
  Request q;
  q.cam_l = l;
  q.cam_r = r;
  q.t = t;
  q.out = out;
  uint64_t tk = 0;
  Status st = s.submit(q, &tk);
  if (code) *code = st.code;
  return st.good() ? tk : 0;
}

static const size_t kBig = (size_t)1 << 30;

// Requests queued within one admission pass form one batch, in FIFO order;
// outputs hold each view's own value; timestamps are ordered.
static void test_fifo_one_batch() {
  FakeExecutor ex(kBig, 5);
  {
    Scheduler s(&ex, kBig, 5.f, 8);
    CHECK(s.start().good());
    Image a(10, 4, 4), b(11, 4, 4);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    std::vector<Out> outs(5, Out(4, 4));
    std::vector<uint64_t> tks;
    s.pause();
    for (int i = 0; i < 5; ++i) tks.push_back(submit(s, i % 2, 1 - i % 2, 0.1f * i, outs[i].p()));
    s.resume();
    for (int i = 0; i < 5; ++i) {
      Timing tm;
      CHECK(wait_ticket(s, tks[i], &tm) == 0);
      CHECK(tm.t_submit <= tm.t_admit && tm.t_admit <= tm.t_launch && tm.t_launch <= tm.t_done);
      const float want = view_value(i % 2 ? 11 : 10, i % 2 ? 10 : 11, 0.1f * i);
      CHECK(outs[i].px[0] == want && outs[i].px.back() == want);
    }
    auto bs = ex.batches();
    CHECK(bs.size() == 1);
    if (bs.size() == 1) {
      CHECK(bs[0].jobs.size() == 5);
      for (int i = 0; i < 5 && i < (int)bs[0].jobs.size(); ++i) CHECK(bs[0].jobs[i].out == outs[i].p());
    }
    // collected tickets are unknown afterwards
    bool done = false;
    CHECK(s.poll(tks[0], nullptr, &done).code == kErrTicket);
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok fifo_one_batch\n");
}

// More requests than max_batch: batches of max_batch in FIFO order; sizes
// mix within a batch, whose slot geometry is its largest view's.
static void test_split_and_resolution() {
  FakeExecutor ex(kBig, 2);
  {
    Scheduler s(&ex, kBig, 5.f, 4);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4), c(3, 8, 8), d(4, 8, 8);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    CHECK(s.register_camera(2, c.px.data(), 8, 8).good());
    CHECK(s.register_camera(3, d.px.data(), 8, 8).good());
    std::vector<Out> small(10, Out(4, 4)), large(3, Out(8, 8));
    std::vector<uint64_t> tks;
    s.pause();
    int si = 0, li = 0;
    const char* order = "SLSSSSLSSSSSL";
    for (const char* o = order; *o; ++o) {
      if (*o == 'S') tks.push_back(submit(s, 0, 1, 0.5f, small[si++].p()));
      else tks.push_back(submit(s, 2, 3, 0.5f, large[li++].p()));
    }
    s.resume();
    for (uint64_t tk : tks) CHECK(wait_ticket(s, tk) == 0);
    auto bs = ex.batches();
    // S0 L0 S1 S2 | S3 S4 L1 S5 | S6..S9 | L2
    CHECK(bs.size() == 4);
    if (bs.size() == 4) {
      CHECK(bs[0].H == 8 && bs[0].W == 8 && bs[0].jobs.size() == 4);
      CHECK(bs[0].jobs[0].out == small[0].p() && bs[0].jobs[0].H == 4 && bs[0].jobs[0].W == 4);
      CHECK(bs[0].jobs[1].out == large[0].p() && bs[0].jobs[1].H == 8 && bs[0].jobs[1].W == 8);
      CHECK(bs[0].jobs[3].out == small[2].p());
      CHECK(bs[1].H == 8 && bs[1].jobs.size() == 4 && bs[1].jobs[2].out == large[1].p() &&
            bs[1].jobs[3].out == small[5].p());
      CHECK(bs[2].H == 4 && bs[2].W == 4 && bs[2].jobs.size() == 4 &&
            bs[2].jobs[0].out == small[6].p() && bs[2].jobs[3].out == small[9].p());
      CHECK(bs[3].H == 8 && bs[3].jobs.size() == 1 && bs[3].jobs[0].out == large[2].p());
    }
    for (auto& o : small) {
      CHECK(o.px[0] == view_value(1, 2, 0.5f));
      CHECK(o.px[3 * 4 * 4 - 1] == view_value(1, 2, 0.5f));
    }
    for (auto& o : large) CHECK(o.px[3 * 8 * 8 - 1] == view_value(3, 4, 0.5f));
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok split_and_resolution\n");
}

// A batch spans at most four sizes: a request of a fifth size waits for the
// next batch while later requests of the four sizes join this one; the slot
// geometry is the largest height and the largest width, which may come from
// different views.
static void test_size_limit_per_batch() {
  FakeExecutor ex(kBig, 2);
  {
    Scheduler s(&ex, kBig, 5.f, 8);
    CHECK(s.start().good());
    const int hs[5] = {4, 6, 8, 4, 10}, ws[5] = {8, 6, 4, 4, 2};
    std::vector<Image> cams;
    for (int k = 0; k < 5; ++k) cams.emplace_back(k + 1, hs[k], ws[k]);
    for (int k = 0; k < 5; ++k) CHECK(s.register_camera(k, cams[k].px.data(), hs[k], ws[k]).good());
    std::vector<Out> outs;
    const int seq[7] = {0, 1, 2, 3, 4, 0, 2};
    for (int k : seq) outs.emplace_back(hs[k], ws[k]);
    std::vector<uint64_t> tks;
    s.pause();
    for (int i = 0; i < 7; ++i) tks.push_back(submit(s, seq[i], seq[i], 0.25f, outs[i].p()));
    s.resume();
    for (uint64_t tk : tks) CHECK(wait_ticket(s, tk) == 0);
    auto bs = ex.batches();
    CHECK(bs.size() == 2);
    if (bs.size() == 2) {
      CHECK(bs[0].jobs.size() == 6 && bs[0].H == 8 && bs[0].W == 8);
      const int want[6] = {0, 1, 2, 3, 5, 6};
      for (int i = 0; i < 6 && i < (int)bs[0].jobs.size(); ++i) CHECK(bs[0].jobs[i].out == outs[want[i]].p());
      CHECK(bs[1].jobs.size() == 1 && bs[1].H == 10 && bs[1].W == 2 && bs[1].jobs[0].out == outs[4].p());
    }
    for (int i = 0; i < 7; ++i) {
      const int k = seq[i];
      CHECK(outs[i].px[3 * hs[k] * ws[k] - 1] == view_value(k + 1, k + 1, 0.25f));
    }
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok size_limit_per_batch\n");
}

// A budget that holds the cameras and one 2-view workspace: batches are
// halved to fit and never overlap; device bytes never exceed the budget.
static void test_budget_admission() {
  const int H = 4, W = 4;
  const size_t cams = 2 * (size_t)H * W * 10, view = (size_t)H * W * 4;
  const size_t budget = cams + 2 * view + view / 2;
  FakeExecutor ex(budget, 3);
  {
    Scheduler s(&ex, budget, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, H, W), b(2, H, W);
    CHECK(s.register_camera(0, a.px.data(), H, W).good());
    CHECK(s.register_camera(1, b.px.data(), H, W).good());
    std::vector<Out> outs(9, Out(H, W));
    std::vector<uint64_t> tks;
    s.pause();
    for (auto& o : outs) tks.push_back(submit(s, 0, 1, 0.25f, o.p()));
    s.resume();
    for (uint64_t tk : tks) CHECK(wait_ticket(s, tk) == 0);
    for (auto& b : ex.batches()) CHECK(b.jobs.size() <= 2);
    CHECK(ex.max_busy() == 1);
    CHECK(ex.peak_bytes() <= budget);
    CHECK(!ex.over_budget_);
    long ad = 0, co = 0, q = 0;
    size_t used = 0;
    CHECK(s.stats(&ad, &co, &q, &used).good());
    CHECK(ad == 9 && co == 9 && q == 0 && used <= budget);
    // a request whose single view can never fit
    Image big(3, 64, 64), big2(4, 64, 64);
    CHECK(s.register_camera(2, big.px.data(), 64, 64).code == kErrBudget);
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok budget_admission\n");
}

// Waves of requests reuse the first slot; concurrent arrivals while a batch
// runs go to a second slot (continuous batching).
static void test_slot_reuse_and_overlap() {
  FakeExecutor ex(kBig, 40);
  {
    Scheduler s(&ex, kBig, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    Out o1(4, 4), o2(4, 4);
    for (int wave = 0; wave < 3; ++wave) CHECK(wait_ticket(s, submit(s, 0, 1, 0.5f, o1.p())) == 0);
    CHECK(ex.slots_created_.load() == 1);
    // second request arrives while the first runs: it does not wait for it
    const uint64_t t1 = submit(s, 0, 1, 0.3f, o1.p());
    std::this_thread::sleep_for(std::chrono::milliseconds(10));
    const uint64_t t2 = submit(s, 1, 0, 0.7f, o2.p());
    Timing m1, m2;
    CHECK(wait_ticket(s, t1, &m1) == 0);
    CHECK(wait_ticket(s, t2, &m2) == 0);
    CHECK(ex.max_busy() == 2);
    CHECK(m2.t_launch < m1.t_done);
    CHECK(o1.px[0] == view_value(1, 2, 0.3f) && o2.px[0] == view_value(2, 1, 0.7f));
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok slot_reuse_and_overlap\n");
}

// A batch whose launch fails reports the failure on each of its tickets
// (then collected); later batches run.
static void test_launch_fault() {
  FakeExecutor ex(kBig, 1);
  {
    Scheduler s(&ex, kBig, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    fault_arm("launch:1");
    Out o1(4, 4), o2(4, 4), o3(4, 4);
    s.pause();
    const uint64_t t1 = submit(s, 0, 1, 0.5f, o1.p());
    const uint64_t t2 = submit(s, 0, 1, 0.5f, o2.p());
    s.resume();
    CHECK(wait_ticket(s, t1) == kErrDevice);
    CHECK(wait_ticket(s, t2) == kErrDevice);
    bool done = false;
    CHECK(s.poll(t1, nullptr, &done).code == kErrTicket);
    CHECK(o1.px[0] == -1.f);  // never written
    CHECK(wait_ticket(s, submit(s, 0, 1, 0.5f, o3.p())) == 0);
    CHECK(o3.px[0] == view_value(1, 2, 0.5f));
    fault_arm(nullptr);
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok launch_fault\n");
}

// Allocation faults: a camera whose allocation fails is not registered; a
// batch whose workspace cannot be allocated, with nothing in flight, fails
// its head request with the allocation's status; nothing leaks.
static void test_alloc_fault() {
  FakeExecutor ex(kBig, 1);
  {
    Scheduler s(&ex, kBig, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4);
    fault_arm("alloc:1");
    CHECK(s.register_camera(0, a.px.data(), 4, 4).code == kErrOom);
    int code = 0;
    Out o(4, 4);
    submit(s, 0, 0, 0.5f, o.p(), &code);
    CHECK(code == kErrArg);  // camera 0 unknown
    fault_arm(nullptr);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    fault_arm("alloc:1");  // the first slot's workspace
    s.pause();
    Out o1(4, 4), o2(4, 4);
    const uint64_t t1 = submit(s, 0, 1, 0.5f, o1.p());
    const uint64_t t2 = submit(s, 0, 1, 0.5f, o2.p());
    s.resume();
    // the 2-view slot fails; the halved 1-view batch gets a slot
    CHECK(wait_ticket(s, t1) == 0);
    CHECK(wait_ticket(s, t2) == 0);
  }
  fault_arm(nullptr);
  CHECK(ex.live_allocs() == 0);
  {
    // one view per batch: a failed workspace with nothing in flight fails
    // the head request, and the next request gets a slot
    Scheduler s(&ex, kBig, 2.f, 1);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    fault_arm("alloc:1");
    s.pause();
    Out o1(4, 4), o2(4, 4);
    const uint64_t t1 = submit(s, 0, 1, 0.5f, o1.p());
    const uint64_t t2 = submit(s, 0, 1, 0.5f, o2.p());
    s.resume();
    CHECK(wait_ticket(s, t1) == kErrOom);
    CHECK(wait_ticket(s, t2) == 0);
    CHECK(o1.px[0] == -1.f && o2.px[0] == view_value(1, 2, 0.5f));
  }
  fault_arm(nullptr);
  CHECK(ex.live_allocs() == 0);
  // every allocation of a fresh scheduler failing in turn
  for (int n = 1; n <= 6; ++n) {
    FakeExecutor ex2(kBig, 1);
    {
      Scheduler s(&ex2, kBig, 2.f, 8);
      CHECK(s.start().good());
      Image a(1, 4, 4), b(2, 4, 4);
      char spec[32];
      std::snprintf(spec, sizeof spec, "alloc:%d", n);
      fault_arm(spec);
      const Status r0 = s.register_camera(0, a.px.data(), 4, 4);
      const Status r1 = s.register_camera(1, b.px.data(), 4, 4);
      CHECK(r0.good() || r0.code == kErrOom);
      CHECK(r1.good() || r1.code == kErrOom);
      if (r0.good() && r1.good()) {
        Out o(4, 4);
        const int c = wait_ticket(s, submit(s, 0, 1, 0.5f, o.p()));
        CHECK(c == 0 || c == kErrOom);
        if (c == 0) CHECK(o.px[0] == view_value(1, 2, 0.5f));
      }
    }
    fault_arm(nullptr);
    CHECK(ex2.live_allocs() == 0);
  }
  std::printf("ok alloc_fault\n");
}

// Argument errors, camera replacement rules, unknown tickets.
static void test_arguments() {
  FakeExecutor ex(kBig, 1);
  {
    Scheduler s(&ex, kBig, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4), c(3, 8, 8), a2(7, 4, 4);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    CHECK(s.register_camera(2, c.px.data(), 8, 8).good());
    CHECK(s.register_camera(0, c.px.data(), 8, 8).code == kErrArg);  // size change
    CHECK(s.register_camera(3, nullptr, 4, 4).code == kErrArg);
    CHECK(s.register_camera(3, a.px.data(), 1, 4).code == kErrArg);
    Out o(4, 4);
    int code = 0;
    submit(s, 0, 2, 0.5f, o.p(), &code);
    CHECK(code == kErrArg);  // sizes differ
    submit(s, 0, 9, 0.5f, o.p(), &code);
    CHECK(code == kErrArg);  // unknown camera
    submit(s, 0, 1, 1.5f, o.p(), &code);
    CHECK(code == kErrArg);
    submit(s, 0, 1, 0.5f, nullptr, &code);
    CHECK(code == kErrArg);
    bool done = false;
    CHECK(s.poll(12345, nullptr, &done).code == kErrTicket);
    // same-size replacement: later views read the new image
    CHECK(s.register_camera(0, a2.px.data(), 4, 4).good());
    CHECK(wait_ticket(s, submit(s, 0, 1, 0.5f, o.p())) == 0);
    CHECK(o.px[0] == view_value(7, 2, 0.5f));
    int h = 0, w = 0;
    CHECK(s.camera_size(2, &h, &w) && h == 8 && w == 8);
    CHECK(!s.camera_size(5, &h, &w));
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok arguments\n");
}

// submit_many: a bad request queues none of them (its index reported); a
// good burst of two sizes is admitted as one batch, in order.
static void test_submit_many() {
  FakeExecutor ex(kBig, 1);
  {
    Scheduler s(&ex, kBig, 2.f, 8);
    CHECK(s.start().good());
    Image a(1, 4, 4), b(2, 4, 4), c(3, 6, 10), d(4, 6, 10);
    CHECK(s.register_camera(0, a.px.data(), 4, 4).good());
    CHECK(s.register_camera(1, b.px.data(), 4, 4).good());
    CHECK(s.register_camera(2, c.px.data(), 6, 10).good());
    CHECK(s.register_camera(3, d.px.data(), 6, 10).good());
    std::vector<Out> outs;
    for (int i = 0; i < 6; ++i) outs.emplace_back(i % 3 == 1 ? 6 : 4, i % 3 == 1 ? 10 : 4);
    std::vector<Request> rs(6);
    for (int i = 0; i < 6; ++i) {
      rs[i].cam_l = i % 3 == 1 ? 2 : 0;
      rs[i].cam_r = i % 3 == 1 ? 3 : 1;
      rs[i].t = 0.125f * i;
      rs[i].out = outs[i].p();
    }
    uint64_t tks[6] = {};
    int bad = -1;
    rs[3].cam_r = 9;  // unknown camera
    CHECK(s.submit_many(rs.data(), 6, tks, &bad).code == kErrArg && bad == 3);
    rs[3].cam_r = 1;
    long adm = 0, comp = 0, queued = 0;
    size_t bytes = 0;
    CHECK(s.stats(&adm, &comp, &queued, &bytes).good() && queued == 0 && adm == 0);
    CHECK(s.submit_many(rs.data(), 0, nullptr, &bad).good());
    CHECK(s.submit_many(rs.data(), 6, tks, &bad).good() && bad == -1);
    for (uint64_t tk : tks) CHECK(wait_ticket(s, tk) == 0);
    auto bs = ex.batches();
    CHECK(bs.size() == 1);
    if (bs.size() == 1) {
      CHECK(bs[0].H == 6 && bs[0].W == 10 && bs[0].jobs.size() == 6);
      for (int i = 0; i < 6 && i < (int)bs[0].jobs.size(); ++i) CHECK(bs[0].jobs[i].out == outs[i].p());
    }
    for (int i = 0; i < 6; ++i) {
      const bool big = i % 3 == 1;
      CHECK(outs[i].px[big ? 3 * 6 * 10 - 1 : 3 * 4 * 4 - 1] ==
            view_value(big ? 3 : 1, big ? 4 : 2, 0.125f * i));
    }
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok submit_many\n");
}

// Several submitting threads at once (ThreadSanitizer's main case): every
// request completes with its own value.
static void test_threads() {
  FakeExecutor ex(kBig, 1);
  {
    Scheduler s(&ex, kBig, 1.f, 16);
    CHECK(s.start().good());
    std::vector<Image> imgs;
    for (int i = 0; i < 4; ++i) imgs.emplace_back(100 + i, 2, 2);
    for (int i = 0; i < 4; ++i) CHECK(s.register_camera(i, imgs[i].px.data(), 2, 2).good());
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int k = 0; k < 4; ++k)
      th.emplace_back([&, k] {
        std::mt19937 rng(k);
        std::vector<Out> outs(100, Out(2, 2));
        std::vector<uint64_t> tks;
        std::vector<float> want;
        for (int i = 0; i < 100; ++i) {
          const int l = rng() % 4, r = rng() % 4;
          const float t = (rng() % 1000) / 1000.f;
          tks.push_back(submit(s, l, r, t, outs[i].p()));
          want.push_back(view_value(100 + l, 100 + r, t));
        }
        for (int i = 0; i < 100; ++i)
          if (wait_ticket(s, tks[i]) != 0 || outs[i].px[0] != want[i]) bad.fetch_add(1);
      });
    for (auto& t : th) t.join();
    CHECK(bad.load() == 0);
  }
  CHECK(ex.live_allocs() == 0);
  std::printf("ok threads\n");
}

int main(int argc, char** argv) {
  fault_arm(nullptr);
  const std::string only = argc > 1 ? argv[1] : "";
  struct T {
    const char* name;
    void (*fn)();
  } tests[] = {{"fifo_one_batch", test_fifo_one_batch},
               {"split_and_resolution", test_split_and_resolution},
               {"size_limit_per_batch", test_size_limit_per_batch},
               {"submit_many", test_submit_many},
               {"budget_admission", test_budget_admission},
               {"slot_reuse_and_overlap", test_slot_reuse_and_overlap},
               {"launch_fault", test_launch_fault},
               {"alloc_fault", test_alloc_fault},
               {"arguments", test_arguments},
               {"threads", test_threads}};
  for (auto& t : tests)
    if (only.empty() || only == t.name) t.fn();
  if (g_failures) {
    std::fprintf(stderr, "%d check(s) failed\n", g_failures);
    return 1;
  }
  std::printf("all passed\n");
  return 0;
}
