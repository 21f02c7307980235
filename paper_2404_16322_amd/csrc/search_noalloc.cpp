// The search on device buffers for callers that cannot allocate device memory: its tables and
// scratch live in one fixed file-scope device array, so the call allocates and frees nothing.
//
// Each device the library runs on holds its own copy of the array for the life of the process.
// Host code never passes the array's name to a kernel or a copy (on the host it stands in for
// the symbol, not for a device address): the device address of each device's copy is looked up
// once per device, with that device current, and only that address is used.
#include "runtime.h"

using namespace ddc;

namespace {

constexpr size_t kStaticBytes = (size_t)64 << 20;   // tables + scratch of one call

__device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mtx;
std::map<int, void *> g_addr;   // device -> address of its copy of `scratch`

// The current device's copy of `scratch` (looked up on the first call on that device).
ddc_status scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_mtx);
  auto it = g_addr.find(dev);
  if (it != g_addr.end()) {
    *out = it->second;
    return DDC_OK;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_err(DDC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  g_addr[dev] = p;
  *out = p;
  return DDC_OK;
}

}  // namespace

extern "C" {

size_t ddc_search_device_noalloc_bytes(void) { return kStaticBytes; }

ddc_status ddc_search_device_noalloc(const ddc_index *ixc, const float *d_queries, int64_t nq,
                                    const int32_t *d_k, int32_t k_all, int32_t k_max,
                                    const int32_t *d_nprobe, int32_t nprobe_all, int32_t nprobe_max,
                                    double significance, ddc_corr mode, const int64_t *d_out_offsets,
                                    int64_t *d_ids, float *d_dists, int64_t *d_counters,
                                    void *hip_stream) {
  ddc_status st = check_device_search(ixc, d_queries, nq, d_k, k_all, k_max, d_nprobe, nprobe_all,
                                      nprobe_max, significance, mode, d_out_offsets, d_ids, d_dists);
  if (st != DDC_OK) return st;
  const int npm = d_nprobe ? nprobe_max : nprobe_all;
  // scratch for one chunk of up to 32768 queries (a larger batch runs chunk after chunk)
  const size_t need = Workspace::kTableBytes + search_scratch_bytes(ixc, nq, npm);
  if (need > kStaticBytes) {
    // the largest batch that fits: the scratch grows linearly in the query count
    const size_t per = search_scratch_bytes(ixc, 2, npm) - search_scratch_bytes(ixc, 1, npm);
    const size_t fixed = search_scratch_bytes(ixc, 1, npm) - per + Workspace::kTableBytes;
    const long long fit = per ? (long long)((kStaticBytes - std::min(fixed, kStaticBytes)) / per) : 0;
    return set_err(DDC_EINVAL,
                   "the allocation-free search needs %zu bytes of scratch for %lld queries (nprobe_max %d, "
                   "nlist %d), more than its fixed %zu; at most about %lld queries fit per call",
                   need, (long long)nq, npm, ixc->nlist, kStaticBytes, fit);
  }
  if (nq == 0) return DDC_OK;
  GUARD_BEGIN
  ddc_index *ix = const_cast<ddc_index *>(ixc);
  DeviceGuard dg(ix->device);
  void *addr = nullptr;
  if ((st = scratch_address(ix->device, &addr)) != DDC_OK) return st;
  const Workspace w{addr, kStaticBytes};
  search_device(ix, d_queries, nq, d_k, k_all, d_k ? k_max : k_all, d_nprobe, nprobe_all, npm,
                significance, mode, d_out_offsets, d_ids, d_dists, d_counters,
                reinterpret_cast<hipStream_t>(hip_stream), nullptr, nullptr, /*may_tune=*/false,
                nullptr, /*stream_scratch=*/false, &w);
  return DDC_OK;
  GUARD_END
}

}  // extern "C"
