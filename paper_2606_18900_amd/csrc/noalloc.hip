// Allocation-free read lookup: the same launches as lz_read_lookup, with the
// request scratch (spans, prefix sums, block slots) taken from one fixed array
// that the library owns in device memory instead of a caller buffer.  For
// callers that cannot allocate device memory per call (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the variable's name to a kernel (that is a host-side stand-in);
// it resolves the device address once per device with hipGetSymbolAddress,
// with that device current, and passes that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lz.h"
#include "lz_internal.h"

int lz_launch_requests(lz_handle* h, const lz_request* d_reqs, const uint32_t* d_n, uint64_t n_max,
                       uint64_t single_off, uint64_t single_len, const int64_t* d_ids,
                       uint8_t* d_out, uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                       uint64_t scratch_len, hipStream_t s);

namespace {

static __device__ __align__(256) uint8_t scratch[LZ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of this device's scratch array, resolved once per device
// (the device must be current).  Called by lz_open, so that the entry point
// itself only reads the cached pointer.
int lz_noalloc_setup(int dev, void** ptr) {
  if (dev < 0 || dev >= kMaxDevices) return lz_fail(LZ_EDEVICE, "device %d outside the supported range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return lz_fail(LZ_EDEVICE, "scratch array address: %s", hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return LZ_OK;
}

extern "C" int lz_read_lookup_noalloc(lz_handle* h, const int64_t* d_ids, uint64_t n, uint8_t* d_out,
                                      uint64_t cap, uint64_t* d_offsets, hipStream_t s) {
  if (!h) return lz_fail(LZ_EINVAL, "lz_read_lookup_noalloc: null handle");
  if (h->av.kind != 1) return lz_fail(LZ_ENOINDEX, "lz_read_lookup_noalloc: archive has no read index");
  if (!n) return LZ_OK;
  if (n > LZ_NOALLOC_MAX_IDS)
    return lz_fail(LZ_ECAPACITY, "lz_read_lookup_noalloc: %llu ids exceed the maximum of %d per call",
                   (unsigned long long)n, LZ_NOALLOC_MAX_IDS);
  if (!d_ids || !d_out || !d_offsets) return lz_fail(LZ_EINVAL, "lz_read_lookup_noalloc: null argument");
  if (cap < n * (uint64_t)h->av.max_record_len)
    return lz_fail(LZ_ECAPACITY, "lz_read_lookup_noalloc: output needs %llu bytes",
                   (unsigned long long)(n * (uint64_t)h->av.max_record_len));
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lz_fail(LZ_EDEVICE, "lz_read_lookup_noalloc: %s", hipGetErrorString(e));
  if (dev != h->dev) return lz_fail(LZ_EINVAL, "lz_read_lookup_noalloc: current device %d is not the handle's %d", dev, h->dev);
  void* p = nullptr;
  const int rc = lz_noalloc_setup(dev, &p);
  if (rc) return rc;
  return lz_launch_requests(h, nullptr, nullptr, n, 0, 0, d_ids, d_out, cap, d_offsets, p,
                            LZ_NOALLOC_SCRATCH_BYTES, s);
}
