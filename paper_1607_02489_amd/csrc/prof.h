// Optional HIP-event timing of kernel classes (launch count, device time,
// algorithmic bytes), read back through emin_profile_collect.
#pragma once
#include "common.h"

namespace emin {
namespace prof {

bool enabled(int kind);
// records a start event on s; returns a token (or -1 when disabled)
int begin(hipStream_t s, int kind, double bytes, double flops);
void end(int token, hipStream_t s);
// a record whose two events the caller hands to a launch that records them
// itself at the kernel's start and end (hipExtLaunchKernel), so the time is
// the kernel's alone; false (events untouched) when the kind is not timed or
// s is capturing
bool begin_launch(hipStream_t s, int kind, double bytes, double flops, hipEvent_t* e0,
                  hipEvent_t* e1);

struct Scope {
  int tok;
  hipStream_t s;
  Scope(hipStream_t s_, int kind, double bytes, double flops = 0.0)
      : tok(enabled(kind) ? begin(s_, kind, bytes, flops) : -1), s(s_) {}
  ~Scope() {
    if (tok >= 0) end(tok, s);
  }
};

}  // namespace prof
}  // namespace emin
