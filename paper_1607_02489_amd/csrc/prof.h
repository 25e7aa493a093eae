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
