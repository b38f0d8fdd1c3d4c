// Staging of kernel descriptors for batched launches.
//
// A per-device ring of pinned host memory and a matching ring of device memory.
// Each request takes the next region of both rings; the host copy is written at
// once and an asynchronous copy moves it to the device on the caller's stream,
// ahead of the kernels that read it; after those kernels are enqueued the caller
// records a fence (an event) on the stream.  When a ring wraps, every fence of the
// lap is waited for, so no region is rewritten while a copy or a kernel of the
// previous lap may still read it.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace ttnn {
namespace {

struct Ring {
  char* host = nullptr;    // pinned
  char* dev = nullptr;
  size_t cap = 0, head = 0;
  std::vector<hipEvent_t> fences;  // recorded after the readers of the current lap
  size_t nfences = 0;              // fences in use this lap (the rest are spare)
};

std::recursive_mutex g_mu;
std::map<int, Ring> g_rings;

constexpr size_t kRingBytes = size_t(8) << 20;
constexpr size_t kAlign = 256;

void drain(Ring& r) {
  for (size_t i = 0; i < r.nfences; ++i) TTNN_HIP(hipEventSynchronize(r.fences[i]));
  r.nfences = 0;
}

}  // namespace

StagingLock::StagingLock() { g_mu.lock(); }
StagingLock::~StagingLock() { g_mu.unlock(); }

void* stage_descriptors(const void* host, size_t bytes, hipStream_t st) {
  std::lock_guard<std::recursive_mutex> lock(g_mu);
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  Ring& r = g_rings[dev];
  const size_t need = (bytes + kAlign - 1) / kAlign * kAlign;
  if (need > r.cap) {                       // first use, or a request larger than the ring
    drain(r);
    if (r.host) TTNN_HIP(hipHostFree(r.host));
    if (r.dev) TTNN_HIP(hipFree(r.dev));
    r.host = nullptr;
    r.dev = nullptr;
    r.cap = std::max(kRingBytes, need);
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, r.cap, hipHostMallocDefault) != hipSuccess || hipMalloc(&d, r.cap) != hipSuccess) {
      (void)hipGetLastError();
      if (h) (void)hipHostFree(h);
      r.cap = 0;
      throw Error{TTNN_E_NOMEM, "descriptor staging ring allocation failed"};
    }
    r.host = static_cast<char*>(h);
    r.dev = static_cast<char*>(d);
    r.head = 0;
  }
  if (r.head + need > r.cap) {              // wrap: the previous lap must be finished
    drain(r);
    r.head = 0;
  }
  char* h = r.host + r.head;
  char* d = r.dev + r.head;
  r.head += need;
  std::memcpy(h, host, bytes);
  TTNN_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
  return d;
}

void fence_descriptors(hipStream_t st) {
  std::lock_guard<std::recursive_mutex> lock(g_mu);
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  Ring& r = g_rings[dev];
  if (r.nfences == r.fences.size()) {
    hipEvent_t e = nullptr;
    TTNN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    r.fences.push_back(e);
  }
  TTNN_HIP(hipEventRecord(r.fences[r.nfences], st));
  ++r.nfences;
}

}  // namespace ttnn
