// Device side of the serving scheduler: runs batches of views of the
// network on HIP streams, over cameras kept resident in device memory.
#pragma once

#include "net.h"
#include "scheduler.h"

namespace ffv {

class HipExecutor : public Executor {
 public:
  explicit HipExecutor(Net* net) : net_(net) {}
  ~HipExecutor() override;
  Status init();
  size_t camera_bytes(int H, int W) const override;
  size_t batch_bytes(int H, int W, int n) const override;
  Status camera_create(int index, const float* image, int H, int W, void** cam) override;
  void camera_destroy(void* cam) override;
  Status slot_create(size_t bytes, void** slot) override;
  Status slot_resize(void* slot, size_t bytes) override;
  void slot_destroy(void* slot) override;
  void slot_wait(void* slot) override;
  Status launch(void* slot, int H, int W, const ViewJob* jobs, int n, void (*done)(void*),
                void* ctx) override;

 private:
  Net* net_;
  CamDev* cam_table_ = nullptr;  // device table, Scheduler::kMaxCams entries
};

}  // namespace ffv
