// Serving scheduler (host-only; no HIP types): continuous batching of
// viewpoint requests over resident cameras under a device-memory admission
// budget. The device side (camera data, batch workspaces, streams, the
// network's launches) sits behind the Executor interface; the library's
// implementation runs the network on HIP streams, and tests drive the same
// scheduler with a host-only executor.
//
// Policy (the paper's multi-user setting: every user asks for the view at
// its own phase between two neighbouring cameras, one network evaluation
// per view):
//   - requests are queued in submission order and admitted once per tick,
//     or as soon as a running batch completes;
//   - a batch holds the queued requests in FIFO order, at most max_batch of
//     them and of at most kMaxSizes distinct resolutions (a request of one
//     more resolution waits for a later batch); the device runs every layer
//     of a batch as one launch over its resolution groups;
//   - a batch runs on a slot (a stream with its own workspace); a free slot
//     that is large enough is reused, else one is grown or created while
//     resident cameras plus all slot workspaces stay within the budget; a
//     batch that does not fit is halved;
//   - batches of consecutive ticks run concurrently on different slots.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "status.h"

namespace ffv {

struct Request {
  int cam_l = 0, cam_r = 0;
  float t = 0.f;
  float* out = nullptr;
  uint64_t tag = 0;
};

struct Timing {
  double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

// One view of a batch: camera table indices, phase, output, and its size.
struct ViewJob {
  int cam_l = 0, cam_r = 0;
  float t = 0.f;
  float* out = nullptr;
  int H = 0, W = 0;
};

// Device side of the scheduler. Every call but launch()'s completion
// callback comes from one thread at a time (the scheduler holds its lock).
class Executor {
 public:
  virtual ~Executor() = default;
  // Device bytes of one resident camera, and of the workspace of a batch of
  // n views whose largest height and width are H and W.
  virtual size_t camera_bytes(int H, int W) const = 0;
  virtual size_t batch_bytes(int H, int W, int n) const = 0;
  // Copy `image` (device, planar [3][H][W]) and build its resident data as
  // entry `index` of the camera table; synchronous. *cam receives a handle.
  virtual Status camera_create(int index, const float* image, int H, int W, void** cam) = 0;
  virtual void camera_destroy(void* cam) = 0;
  // A slot: a stream and a workspace of `bytes`.
  virtual Status slot_create(size_t bytes, void** slot) = 0;
  // Replace the workspace by one of `bytes` (old contents dead). On failure
  // the slot holds no workspace (0 bytes).
  virtual Status slot_resize(void* slot, size_t bytes) = 0;
  virtual void slot_destroy(void* slot) = 0;
  // Block until the work queued on the slot is done.
  virtual void slot_wait(void* slot) = 0;
  // Queue a batch of n views (each of its own size; H x W the largest
  // height and width among them) on the slot. On success, done(ctx)
  // runs exactly once, on any thread and without blocking, after the
  // outputs are written. On failure nothing of the batch is left running
  // and done is not called.
  virtual Status launch(void* slot, int H, int W, const ViewJob* jobs, int n, void (*done)(void*),
                        void* ctx) = 0;
};

class Scheduler {
 public:
  static constexpr int kMaxCams = 1024;
  static constexpr int kMaxSizes = 4;  // resolutions per batch
  Scheduler(Executor* ex, size_t budget, float tick_ms, int max_batch);
  // Stops admitting, waits for the batches in flight, frees slots and
  // cameras. Tickets never admitted are dropped.
  ~Scheduler();
  Status start();
  // Register camera `id` (or replace it by an image of the same size, once
  // the batches in flight are done).
  Status register_camera(int id, const float* image, int H, int W);
  Status submit(const Request& r, uint64_t* ticket);
  // Queue n requests at once: all are checked first and none is queued if
  // one fails (its index in *bad when non-null); the queue takes them in
  // order under one lock, so one admission sees all of them.
  Status submit_many(const Request* rs, int n, uint64_t* tickets, int* bad);
  // *done = false while queued or running. Once finished the ticket is
  // collected: *done = true with the timing, or the status of a failed batch.
  Status poll(uint64_t ticket, Timing* timing, bool* done);
  Status stats(long* admitted, long* completed, long* queued, size_t* bytes_in_use);
  // Size of a registered camera (false when unknown).
  bool camera_size(int id, int* H, int* W);
  // Stop admitting batches and wait until none is in flight; camera
  // registration waits too. Nestable; resume() undoes one pause(). Used
  // around calls that change the network's state (tile tuning, FP8
  // calibration, profiling), so no batch runs while they do.
  void pause();
  void resume();

 private:
  Status check_locked(const Request& r, int* H, int* W) const;
  uint64_t enqueue_locked(const Request& r, int H, int W);
  struct Camera {
    int H = 0, W = 0;
    void* handle = nullptr;
    int index = -1;  // entry in the camera table
  };
  struct Ticket {
    Request req;
    int H = 0, W = 0;
    Timing tm;
    // 0 queued, 1 admitted, 2 done, 3 failed (status in err). 2 is stored
    // by the completion callback (release) after tm.t_done, without the lock.
    std::atomic<int> state{0};
    Status err;
  };
  struct Slot {
    void* h = nullptr;
    size_t bytes = 0;
    std::atomic<bool> busy{false};
    std::vector<Ticket*> tickets;  // written before launch, read by the callback
  };
  struct Done {
    Scheduler* s;
    Slot* slot;  // stable: slots are never moved or freed while serving
  };
  static void on_done(void* p);
  void loop();
  void admit_and_launch();  // called with mu_ held
  void fail_tickets(const std::vector<Ticket*>& tks, const Status& st);
  bool any_busy() const;

  Executor* ex_;
  size_t budget_;
  float tick_ms_;
  int max_batch_;
  std::thread thr_;
  std::mutex mu_;
  std::condition_variable cv_;
  bool stop_ = false;
  int paused_ = 0;
  std::map<int, Camera> cams_;
  std::vector<int> free_cam_index_;
  size_t resident_bytes_ = 0;
  size_t slot_bytes_ = 0;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, Ticket> tickets_;  // nodes are stable: callbacks hold Ticket*
  uint64_t next_ticket_ = 1;
  std::vector<std::unique_ptr<Slot>> slots_;
  std::vector<std::unique_ptr<Done>> done_ctx_;
  long n_admitted_ = 0;
  std::atomic<long> n_completed_{0};
};

// RAII pause of a scheduler (no-op for nullptr).
class ServingPause {
 public:
  explicit ServingPause(Scheduler* s) : s_(s) {
    if (s_) s_->pause();
  }
  ~ServingPause() {
    if (s_) s_->resume();
  }
  ServingPause(const ServingPause&) = delete;
  ServingPause& operator=(const ServingPause&) = delete;

 private:
  Scheduler* s_;
};

double now_seconds();

}  // namespace ffv
