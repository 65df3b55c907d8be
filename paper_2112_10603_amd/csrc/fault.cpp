// Fault injection hook (see fault.h).
#include "fault.h"

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

namespace ffv {

namespace {

struct FaultState {
  std::mutex mu;
  bool loaded = false;
  long alloc_at = 0, launch_at = 0;  // 0: never
  long alloc_n = 0, launch_n = 0;    // occurrences so far
};

FaultState& state() {
  static FaultState s;
  return s;
}

void parse(FaultState& s, const char* spec) {
  s.alloc_at = s.launch_at = 0;
  s.alloc_n = s.launch_n = 0;
  if (!spec) return;
  std::string t(spec);
  size_t pos = 0;
  while (pos < t.size()) {
    size_t end = t.find(',', pos);
    if (end == std::string::npos) end = t.size();
    const std::string item = t.substr(pos, end - pos);
    const size_t colon = item.find(':');
    if (colon != std::string::npos) {
      const long n = std::strtol(item.c_str() + colon + 1, nullptr, 10);
      const std::string kind = item.substr(0, colon);
      if (n > 0 && kind == "alloc") s.alloc_at = n;
      if (n > 0 && kind == "launch") s.launch_at = n;
    }
    pos = end + 1;
  }
}

}  // namespace

void fault_arm(const char* spec) {
  FaultState& s = state();
  std::lock_guard<std::mutex> lk(s.mu);
  parse(s, spec);
  s.loaded = true;
}

bool fault_hit(const char* kind) {
  FaultState& s = state();
  std::lock_guard<std::mutex> lk(s.mu);
  if (!s.loaded) {
    parse(s, std::getenv("FFV_FAULT"));
    s.loaded = true;
  }
  if (std::strcmp(kind, "alloc") == 0) return s.alloc_at > 0 && ++s.alloc_n == s.alloc_at;
  if (std::strcmp(kind, "launch") == 0) return s.launch_at > 0 && ++s.launch_n == s.launch_at;
  return false;
}

}  // namespace ffv
