// Fault injection for tests of the error paths (host-only).
//
// FFV_FAULT="alloc:N" makes the N-th device allocation of the process
// (counted from the first check) report out-of-memory; "launch:N" makes the
// N-th serving batch launch fail before anything is queued. Several
// entries may be joined with ','. The hook only makes host calls return an
// error: no device work is issued for a failed step.
#pragma once

namespace ffv {

// True when this occurrence of `kind` ("alloc" or "launch") must fail.
bool fault_hit(const char* kind);
// Replace the active fault spec (the environment is read only if this was
// never called); resets the counters. nullptr or "" disarms.
void fault_arm(const char* spec);

}  // namespace ffv
