// A stand-in for the HIP runtime calls the library's host code makes, for
// checking that code on a machine without a GPU (see hostcheck.h).
//
// Model.  Streams carry vector clocks: an operation enqueued on stream s
// advances s's own entry; an event records the clock of its stream; a wait
// merges the event's clock into the waiting stream's.  The host's knowledge
// of finished work is a clock too, advanced by stream and event
// synchronisation.  Rules checked (each a requirement of the HIP / CUDA
// stream-capture and graph model, or of this library's own contract):
//  - every handle passed in is a live object of the right kind;
//  - a capture forks only through events recorded inside it, every forked
//    stream joins back before the capture ends, and nothing inside a capture
//    synchronises, allocates or waits on an event recorded outside it;
//  - an event recorded inside a capture is never waited on or synchronised
//    outside it;
//  - an executable graph is destroyed only once the host knows that all of
//    its launches have finished;
//  - device memory is freed once, and only memory the stub handed out.
// Elapsed times are deterministic pseudo-random values, so the autotuner's
// choices vary from run to run of the driver's scenarios.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "hostcheck.h"

namespace {

constexpr uint32_t kStream = 0x5354524d, kEvent = 0x45564e54, kGraph = 0x47525048, kExec = 0x45584543;

struct Capture;

struct Stream {
  uint32_t magic = kStream;
  int id = 0;
  std::vector<uint64_t> clock;
  Capture* cap = nullptr;
  long cap_ops = 0;     // operations recorded into the capture on this stream
  long joined_at = -1;  // cap_ops value at which the origin last joined this stream's work
};

struct Event {
  uint32_t magic = kEvent;
  bool recorded = false;
  std::vector<uint64_t> clock;  // outside captures
  Capture* cap = nullptr;       // recorded inside this capture (still open)
  Stream* cap_stream = nullptr;
  long cap_pos = 0;
  bool captured_ever = false;   // last record happened inside a capture
};

struct Capture {
  Stream* origin;
  std::set<Stream*> members;
  long nodes = 0;
};

struct Graph {
  uint32_t magic = kGraph;
  long nodes = 0;
};

struct Exec {
  uint32_t magic = kExec;
  long nodes = 0;
  std::map<int, uint64_t> last_launch;  // stream id -> sequence number of the latest launch
};

struct State {
  std::vector<Stream*> streams;  // by id; null once destroyed
  Stream null_stream;
  std::vector<uint64_t> host;    // host-known finished work per stream
  std::map<uintptr_t, size_t> allocs;
  std::map<const void*, size_t> var_sizes;   // registered device variables
  std::map<const void*, void*> var_storage;  // their stand-in storage
  std::set<void*> objects;       // live streams / events / graphs / execs
  struct Copy {                  // an asynchronous copy the host has not yet seen finish
    void* dst;
    const void* src;
    size_t bytes;
    std::vector<uint64_t> clock;
  };
  std::vector<Copy> copies;
  hc::Counts counts;
  uint64_t rng = 0x9e3779b97f4a7c15ull;
  State() {
    null_stream.id = 0;
    streams.push_back(&null_stream);
  }
};

State& S() {
  static State* s = new State();
  return *s;
}

uint64_t& at(std::vector<uint64_t>& v, int i) {
  if (static_cast<int>(v.size()) <= i) v.resize(i + 1, 0);
  return v[i];
}

void merge(std::vector<uint64_t>& into, const std::vector<uint64_t>& from) {
  if (into.size() < from.size()) into.resize(from.size(), 0);
  for (size_t i = 0; i < from.size(); ++i) into[i] = std::max(into[i], from[i]);
}

Stream* stream_of(hipStream_t h, const char* call) {
  if (h == nullptr) return &S().null_stream;
  Stream* s = reinterpret_cast<Stream*>(h);
  if (!S().objects.count(s) || s->magic != kStream) hc::violation("%s: not a live stream (%p)", call, (void*)h);
  return s;
}

Event* event_of(hipEvent_t h, const char* call) {
  Event* e = reinterpret_cast<Event*>(h);
  if (h == nullptr || !S().objects.count(e) || e->magic != kEvent)
    hc::violation("%s: not a live event (%p)", call, (void*)h);
  return e;
}

// With HOSTCHECK_TRACE set, every stream operation is printed.
bool tracing() {
  static const bool on = std::getenv("HOSTCHECK_TRACE") != nullptr;
  return on;
}

// One operation in the order of stream s.
void enqueue(Stream* s) {
  if (s->cap) {
    s->cap->nodes++;
    s->cap_ops++;
    S().counts.captured_nodes++;
    return;
  }
  at(s->clock, s->id)++;
  if (tracing()) std::fprintf(stderr, "  stream %d op %llu\n", s->id, (unsigned long long)s->clock[s->id]);
}

bool host_knows(const std::vector<uint64_t>& clock) {
  std::vector<uint64_t>& h = S().host;
  for (size_t i = 0; i < clock.size(); ++i)
    if (clock[i] > (i < h.size() ? h[i] : 0)) return false;
  return true;
}

// Asynchronous copies move their bytes at once (so later stub launches see
// them) and again once the host has waited for them: a host buffer released
// or reused before that wait is read or written after its end of life, which
// the sanitizer reports.
void settle_copies() {
  auto& v = S().copies;
  for (size_t i = 0; i < v.size();) {
    if (host_knows(v[i].clock)) {
      std::memmove(v[i].dst, v[i].src, v[i].bytes);
      v.erase(v.begin() + static_cast<std::ptrdiff_t>(i));
    } else {
      ++i;
    }
  }
}

void* new_alloc(size_t bytes) {
  const size_t b = std::max<size_t>(256, (bytes + 255) / 256 * 256);
  void* p = std::aligned_alloc(256, b);
  if (p == nullptr) return nullptr;
  std::memset(p, 0xA5, b);  // the library must not rely on fresh memory being zero
  S().allocs[reinterpret_cast<uintptr_t>(p)] = bytes;
  S().counts.allocations++;
  return p;
}

}  // namespace

namespace hc {

void violation(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "hostcheck VIOLATION: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
  std::abort();
}

void need(const void* p, size_t bytes, const char* what) {
  if (p == nullptr) violation("%s: null buffer", what);
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto& m = S().allocs;
  auto it = m.upper_bound(a);
  if (it == m.begin()) violation("%s: %p is not in a stub allocation", what, p);
  --it;
  if (a < it->first || a + bytes > it->first + it->second || a + bytes < a)
    violation("%s: [%p, +%zu) is outside its allocation [%p, +%zu)", what, p, bytes,
              reinterpret_cast<void*>(it->first), it->second);
}

void kernel_launch(hipStream_t stream, const char* name) {
  Stream* s = stream_of(stream, name);
  if (!s->cap) S().counts.launches++;
  enqueue(s);
}

Counts counts() { return S().counts; }

long live_objects() {
  long n = static_cast<long>(S().allocs.size() - S().var_storage.size());
  for (void* o : S().objects)
    if (static_cast<Event*>(o)->magic != kEvent) ++n;  // the timing profiler keeps a pool of events
  return n;
}

}  // namespace hc

extern "C" {

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}

hipError_t hipSetDevice(int d) {
  if (d != 0) hc::violation("hipSetDevice(%d): the stub has one device", d);
  return hipSuccess;
}

hipError_t hipGetLastError(void) { return hipSuccess; }

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stub error"; }

hipError_t hipStreamCreateWithFlags(hipStream_t* out, unsigned int) {
  Stream* s = new Stream();
  s->id = static_cast<int>(S().streams.size());
  S().streams.push_back(s);
  S().objects.insert(s);
  *out = reinterpret_cast<hipStream_t>(s);
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t h) {
  Stream* s = stream_of(h, "hipStreamDestroy");
  if (s == &S().null_stream) hc::violation("hipStreamDestroy of the default stream");
  if (s->cap) hc::violation("hipStreamDestroy of a stream inside a capture");
  S().streams[s->id] = nullptr;
  S().objects.erase(s);
  delete s;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t h) {
  if (tracing()) std::fprintf(stderr, "hipStreamSynchronize %p\n", (void*)h);
  Stream* s = stream_of(h, "hipStreamSynchronize");
  if (s->cap) hc::violation("hipStreamSynchronize on a capturing stream");
  merge(S().host, s->clock);
  settle_copies();
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* out, unsigned) {
  Event* e = new Event();
  S().objects.insert(e);
  *out = reinterpret_cast<hipEvent_t>(e);
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* out) { return hipEventCreateWithFlags(out, 0); }

hipError_t hipEventDestroy(hipEvent_t h) {
  Event* e = event_of(h, "hipEventDestroy");
  if (e->cap) hc::violation("hipEventDestroy of an event recorded in a capture that is still open");
  S().objects.erase(e);
  delete e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t h, hipStream_t st) {
  if (tracing()) std::fprintf(stderr, "hipEventRecord %p on %p\n", (void*)h, (void*)st);
  Event* e = event_of(h, "hipEventRecord");
  Stream* s = stream_of(st, "hipEventRecord");
  enqueue(s);
  e->recorded = true;
  if (s->cap) {
    e->cap = s->cap;
    e->cap_stream = s;
    e->cap_pos = s->cap_ops;
    e->captured_ever = true;
  } else {
    e->cap = nullptr;
    e->captured_ever = false;
    e->clock = s->clock;
  }
  return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t h, unsigned int) {
  Stream* t = stream_of(st, "hipStreamWaitEvent");
  Event* e = event_of(h, "hipStreamWaitEvent");
  if (!e->recorded) return hipSuccess;  // waiting on a never-recorded event is a no-op
  if (e->cap) {
    if (t->cap == nullptr) {  // t forks into the capture
      t->cap = e->cap;
      t->cap_ops = 0;
      t->joined_at = -1;
      e->cap->members.insert(t);
    } else if (t->cap != e->cap) {
      hc::violation("hipStreamWaitEvent: the stream and the event belong to different captures");
    }
    // the origin now depends on e's stream up to e's position: that stream has
    // joined back if nothing was recorded on it after e
    if (t == e->cap->origin && e->cap_stream != t && e->cap_pos == e->cap_stream->cap_ops)
      e->cap_stream->joined_at = e->cap_pos;
    enqueue(t);
    return hipSuccess;
  }
  if (e->captured_ever) hc::violation("hipStreamWaitEvent on an event recorded in a capture that has ended");
  if (t->cap) hc::violation("hipStreamWaitEvent inside a capture on an event recorded outside it");
  merge(t->clock, e->clock);
  enqueue(t);
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t h) {
  if (tracing()) std::fprintf(stderr, "hipEventSynchronize %p\n", (void*)h);
  Event* e = event_of(h, "hipEventSynchronize");
  if (e->cap || e->captured_ever) hc::violation("hipEventSynchronize on an event recorded in a capture");
  if (e->recorded) merge(S().host, e->clock);
  settle_copies();
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  Event* s = event_of(a, "hipEventElapsedTime");
  Event* t = event_of(b, "hipEventElapsedTime");
  if (!s->recorded || !t->recorded) hc::violation("hipEventElapsedTime on an event never recorded");
  if (s->captured_ever || t->captured_ever) hc::violation("hipEventElapsedTime on an event recorded in a capture");
  if (!host_knows(t->clock)) hc::violation("hipEventElapsedTime before the stop event is known to be complete");
  uint64_t& r = S().rng;
  r = r * 6364136223846793005ull + 1442695040888963407ull;
  *ms = 1.0f + static_cast<float>((r >> 33) % 1000) / 100.0f;
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
  Stream* s = stream_of(st, "hipStreamBeginCapture");
  if (s == &S().null_stream) hc::violation("hipStreamBeginCapture on the default stream");
  if (s->cap) hc::violation("hipStreamBeginCapture on a stream already capturing");
  Capture* c = new Capture();
  c->origin = s;
  c->members.insert(s);
  s->cap = c;
  s->cap_ops = 0;
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* out) {
  Stream* s = stream_of(st, "hipStreamEndCapture");
  Capture* c = s->cap;
  if (c == nullptr || c->origin != s) hc::violation("hipStreamEndCapture on a stream that did not begin a capture");
  for (Stream* m : c->members)
    if (m != s && m->joined_at != m->cap_ops)
      hc::violation("hipStreamEndCapture: stream %d forked into the capture and did not join back", m->id);
  for (Stream* m : c->members) m->cap = nullptr;
  // events recorded in this capture stay marked as captured (captured_ever)
  for (void* o : S().objects) {
    Event* e = static_cast<Event*>(o);
    if (e->magic == kEvent && e->cap == c) e->cap = nullptr;
  }
  Graph* g = new Graph();
  g->nodes = c->nodes;
  delete c;
  S().objects.insert(g);
  *out = reinterpret_cast<hipGraph_t>(g);
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* out, hipGraph_t h, hipGraphNode_t*, char*, size_t) {
  Graph* g = reinterpret_cast<Graph*>(h);
  if (!S().objects.count(g) || g->magic != kGraph) hc::violation("hipGraphInstantiate: not a live graph");
  Exec* x = new Exec();
  x->nodes = g->nodes;
  S().objects.insert(x);
  S().counts.graphs++;
  *out = reinterpret_cast<hipGraphExec_t>(x);
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t h, hipStream_t st) {
  if (tracing()) std::fprintf(stderr, "hipGraphLaunch %p\n", (void*)h);
  Exec* x = reinterpret_cast<Exec*>(h);
  if (!S().objects.count(x) || x->magic != kExec) hc::violation("hipGraphLaunch: not a live executable graph");
  Stream* s = stream_of(st, "hipGraphLaunch");
  if (s->cap) hc::violation("hipGraphLaunch inside a capture");
  enqueue(s);
  x->last_launch[s->id] = at(s->clock, s->id);
  S().counts.graph_launches++;
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t h) {
  if (tracing()) std::fprintf(stderr, "hipGraphExecDestroy %p\n", (void*)h);
  Exec* x = reinterpret_cast<Exec*>(h);
  if (!S().objects.count(x) || x->magic != kExec) hc::violation("hipGraphExecDestroy: not a live executable graph");
  for (auto& [sid, seq] : x->last_launch) {
    const uint64_t known = sid < static_cast<int>(S().host.size()) ? S().host[sid] : 0;
    if (known < seq)
      hc::violation("hipGraphExecDestroy while a launch of it on stream %d may still run (launch %llu, host "
                    "knows %llu)", sid, (unsigned long long)seq, (unsigned long long)known);
  }
  S().objects.erase(x);
  delete x;
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t h) {
  Graph* g = reinterpret_cast<Graph*>(h);
  if (!S().objects.count(g) || g->magic != kGraph) hc::violation("hipGraphDestroy: not a live graph");
  S().objects.erase(g);
  delete g;
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t bytes) {
  for (Stream* s : S().streams)
    if (s && s->cap) hc::violation("hipMalloc while a capture is open");
  *p = new_alloc(bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t st) {
  Stream* s = stream_of(st, "hipMallocAsync");
  if (s->cap) hc::violation("hipMallocAsync inside a capture");
  enqueue(s);
  *p = new_alloc(bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

// Pinned host memory: the GPU may write it, so it is tracked like a device
// allocation (kernels' parameters are checked against it) and released with
// hipHostFree only.
std::set<void*>& host_allocs() {
  static std::set<void*>* s = new std::set<void*>();
  return *s;
}

hipError_t hipFree(void* p) {
  if (p == nullptr) return hipSuccess;
  if (host_allocs().count(p)) hc::violation("hipFree of %p, a pinned host allocation (hipHostFree releases it)", p);
  auto it = S().allocs.find(reinterpret_cast<uintptr_t>(p));
  if (it == S().allocs.end()) hc::violation("hipFree of %p, which is not a live stub allocation", p);
  settle_copies();
  const uintptr_t lo = it->first, hi = it->first + it->second;
  for (const auto& c : S().copies) {
    const uintptr_t d = reinterpret_cast<uintptr_t>(c.dst), r = reinterpret_cast<uintptr_t>(c.src);
    if ((d >= lo && d < hi) || (r >= lo && r < hi))
      hc::violation("hipFree of %p while an asynchronous copy into or out of it may still run", p);
  }
  S().allocs.erase(it);
  std::free(p);
  return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = new_alloc(bytes);
  if (*p) host_allocs().insert(*p);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipHostFree(void* p) {
  if (p == nullptr) return hipSuccess;
  if (!host_allocs().erase(p)) hc::violation("hipHostFree of %p, which is not a live pinned allocation", p);
  return hipFree(p);
}

hipError_t hipFreeAsync(void* p, hipStream_t st) {
  Stream* s = stream_of(st, "hipFreeAsync");
  if (s->cap) hc::violation("hipFreeAsync inside a capture");
  enqueue(s);
  return hipFree(p);
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  for (Stream* s : S().streams)
    if (s && s->cap) hc::violation("hipMemcpy while a capture is open");
  if (kind != hipMemcpyHostToDevice) hc::violation("hipMemcpy: only host-to-device copies are modelled");
  hc::need(dst, bytes, "hipMemcpy destination");
  // synchronous: every stream's queued work is done (the legacy stream's semantics)
  for (Stream* s : S().streams)
    if (s) merge(S().host, s->clock);
  settle_copies();
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st) {
  Stream* s = stream_of(st, "hipMemcpyAsync");
  if (s->cap) hc::violation("hipMemcpyAsync inside a capture (not modelled)");
  if (kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) hc::need(dst, bytes, "hipMemcpyAsync destination");
  if (kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) hc::need(src, bytes, "hipMemcpyAsync source");
  if (kind != hipMemcpyHostToDevice && kind != hipMemcpyDeviceToHost && kind != hipMemcpyDeviceToDevice)
    hc::violation("hipMemcpyAsync: copy kind %d is not modelled", static_cast<int>(kind));
  enqueue(s);
  std::memmove(dst, src, bytes);
  S().copies.push_back(State::Copy{dst, src, bytes, s->clock});
  return hipSuccess;
}

hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size, hipDeviceptr_t p) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto& m = S().allocs;
  auto it = m.upper_bound(a);
  if (it == m.begin()) return hipErrorInvalidValue;
  --it;
  if (a >= it->first + std::max<size_t>(it->second, 1)) return hipErrorInvalidValue;
  *base = reinterpret_cast<hipDeviceptr_t>(it->first);
  *size = it->second;
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** out, const void* symbol) {
  auto& st = S();
  auto v = st.var_storage.find(symbol);
  if (v == st.var_storage.end()) {
    auto sz = st.var_sizes.find(symbol);
    if (sz == st.var_sizes.end()) hc::violation("hipGetSymbolAddress of an unregistered symbol");
    void* p = new_alloc(sz->second);
    if (p == nullptr) return hipErrorOutOfMemory;
    v = st.var_storage.emplace(symbol, p).first;
  }
  *out = v->second;
  return hipSuccess;
}

// ---- module registration emitted by the HIP compiler for device variables ----
void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}

void __hipUnregisterFatBinary(void**) {}

void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) { S().var_sizes[var] = size; }

void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*,
                           int*) {}

}  // extern "C"
