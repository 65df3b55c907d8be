// Status value of the library's internal calls (host-only; no HIP types).
// `code` uses the ffv_status values of include/ffv.h.
#pragma once

#include <string>

namespace ffv {

enum : int {
  kOk = 0,
  kErrArg = -1,
  kErrOom = -2,
  kErrBudget = -3,
  kErrDevice = -4,
  kErrWeights = -5,
  kErrTicket = -6,
  kErrState = -7
};

struct Status {
  int code = 0;  // ffv_status value
  std::string msg;
  static Status ok() { return Status(); }
  static Status err(int c, const std::string& m) {
    Status s;
    s.code = c;
    s.msg = m;
    return s;
  }
  bool good() const { return code == 0; }
};

}  // namespace ffv
