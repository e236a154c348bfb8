// Host-code checks of the structure-tensor library on a machine without a GPU.
//
// The library's host translation units (validation, planning, the pass
// sequence, chunk batches and their autotuner, the surrogate's host side) are
// compiled for the host only, with AddressSanitizer and UBSan, and linked
// against hip_stub.cpp instead of the HIP runtime.  The stub keeps every
// stream, event, graph and allocation as a heap record, and checks each call
// against the rules of the HIP programming model that the library relies on
// (see hip_stub.cpp).  The kernel launch functions are replaced by
// stub_kernels.cpp, which checks every launch's parameters against the
// buffers the kernel would read and write.  Any violation prints a message
// and aborts; ASan and UBSan catch memory and undefined-behaviour errors of
// the host code itself.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hc {

// Aborts with a message (a broken rule of the programming model, or a launch
// that would access memory outside its buffers).
[[noreturn]] void violation(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// [p, p + bytes) must lie inside one live allocation of the stub.
void need(const void* p, size_t bytes, const char* what);

// Records a kernel launch on `stream` (ordering, capture membership).
void kernel_launch(hipStream_t stream, const char* name);

// Counters for the driver's report.
struct Counts {
  long launches = 0;        // kernels enqueued outside captures
  long captured_nodes = 0;  // operations recorded into graphs
  long graphs = 0;          // graphs instantiated
  long graph_launches = 0;
  long allocations = 0;
};
Counts counts();

// Live objects left (streams, graphs, executable graphs, allocations),
// excluding the default stream, the library-held scratch arrays and events
// (the library's timing profiler keeps a pool of events for the process).
long live_objects();

}  // namespace hc
