// kdt_noalloc.hip -- kNN for callers that cannot allocate device memory
// (work captured into a HIP graph, serving loops, harnesses that forbid
// allocation).
//
// kdt_knn takes one kind of scratch on the k <= KDT_MAX_K path: the query
// order (Hilbert or leaf keys, their sorted copy, two index arrays and the
// radix sort's temporary storage).  Here that scratch lives in `scratch`, a
// file-scope device array that every GPU the library runs on holds until the
// process ends.  Its device address is looked up once per device, with that
// device current, and only that address is handed to kernels and library
// calls: in host code `scratch` names a host-side stand-in, not device memory.
//
// Calls on one GPU share its array and leave their contents in it; nothing
// here has to start at zero (every key and index is written before it is
// read).  Calls that overlap on one GPU race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kdt_query.h"

namespace kdt {
namespace {

constexpr size_t kScratchBytes = KDT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DeviceScratch {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
DeviceScratch g_scratch[kMaxDevices];

// The device address of `scratch` on device `dev` (current), looked up on
// the first call for that device.
kdt_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    kdt_set_error("kdt_knn_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    return KDT_EUNSUPPORTED;
  }
  DeviceScratch& s = g_scratch[dev];
  std::call_once(s.once, [&s] {
    s.err = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch));
    if (s.err != hipSuccess) s.ptr = nullptr;
  });
  if (s.err != hipSuccess || !s.ptr) {
    kdt_set_error("kdt_knn_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(s.err));
    return KDT_EDEVICE;
  }
  *out = s.ptr;
  return KDT_OK;
}

}  // namespace
}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_knn_noalloc(const kdt_tree* tree, const float* d_q, int64_t nq,
                                      int32_t k, int32_t* d_idx, float* d_d2, int32_t kth_only,
                                      const kdt_query_opts* opts, hipStream_t stream) {
  kdt_clear_error();
  if (refuse_f64(tree, "kdt_knn_noalloc")) return KDT_EUNSUPPORTED;
  KnnArgs a;
  const kdt_status chk = knn_check(tree, d_q, nq, k, d_d2, kth_only, opts, "kdt_knn_noalloc", &a);
  if (chk != KDT_OK || a.empty) return chk;
  if (k > KDT_MAX_K) {
    kdt_set_error("kdt_knn_noalloc: k=%d above %d (larger k sorts per-query balls, which "
                  "allocates: use kdt_knn)", k, KDT_MAX_K);
    return KDT_EUNSUPPORTED;
  }
  if (a.period) {
    kdt_set_error("kdt_knn_noalloc: periodic boundaries are not supported (use kdt_knn)");
    return KDT_EUNSUPPORTED;
  }
  const bool sorts = d_q && !a.given && a.sort_q && nq > 1;
  if (sorts && nq > KDT_NOALLOC_MAX_SORTED) {
    kdt_set_error("kdt_knn_noalloc: %lld queries to order, at most %d fit the scratch "
                  "(pass sort_queries = 0 or an order from kdt_query_order)",
                  (long long)nq, KDT_NOALLOC_MAX_SORTED);
    return KDT_ECAPACITY;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    kdt_set_error("kdt_knn_noalloc: hipGetDevice failed");
    return KDT_EDEVICE;
  }
  if (dev != tree->device) {
    kdt_set_error("kdt_knn_noalloc: the tree lives on device %d, device %d is current",
                  tree->device, dev);
    return KDT_EINVAL;
  }
  void* ws = nullptr;
  const kdt_status st = scratch_on(dev, &ws);
  if (st != KDT_OK) return st;
  return knn_in_workspace(tree, d_q, nq, k, d_idx, d_d2, kth_only, a, ws, kScratchBytes, stream);
}
