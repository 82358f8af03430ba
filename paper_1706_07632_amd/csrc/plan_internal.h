// Internal interface of the plan object for the entry point that binds a
// plan to the library's own device array (noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "mgwr.h"

namespace mgwr {

// What a plan is bound to: its workspace, stream, device and network.
struct PlanBinding {
  bool bound;
  int device;
  unsigned char* ws;
  size_t bytes;
  hipStream_t stream;
  mgwr_net* net;
};

PlanBinding plan_binding(const mgwr_plan* pl);
// Points the plan back at a binding it had before (no device work: the old
// workspace still holds its packed image).
void restore_binding(mgwr_plan* pl, const PlanBinding& b);
// Drops the plan's network (its slice rows live in the old workspace).
void detach_network(mgwr_plan* pl);
size_t plan_workspace_bytes(const mgwr_plan* pl);

}  // namespace mgwr
