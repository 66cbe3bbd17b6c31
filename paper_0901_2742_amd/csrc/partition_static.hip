// sad_partition_noalloc: the regular-sampling partition (Section 2.3.2, steps
// 7-10) with its scratch in a static device array instead of library or
// caller workspace, for callers that cannot allocate device memory.  The
// kernels and the scratch layout are those of sad_partition.
#include <mutex>

#include "sad_internal.h"

namespace sad {

// Largest scratch the static array holds: 32 MiB covers the partition of
// 200000 ids into 1024 buckets (about 29.2 MiB: the p(p-1) regular samples
// twice, per-block bucket counts, the chunk order).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in; the device address comes
// from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int32_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return report_error(SAD_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= 64) return report_error(SAD_E_DEVICE, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return report_error(SAD_E_DEVICE,
                          std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SAD_OK;
}

}  // namespace sad

using namespace sad;

extern "C" int32_t sad_partition_noalloc(const sad_seqs* seqs, const uint64_t* d_key,
                                         const sad_params* prm, uint64_t* d_pivot_key,
                                         int32_t* d_pivot_id, int32_t* d_bucket,
                                         int32_t* d_bucket_off, int32_t* d_members,
                                         hipStream_t stream) {
  if (!seqs || !prm) return report_error(SAD_E_INVAL, "null argument");
  if (prm->p < 1) return report_error(SAD_E_INVAL, "p must be >= 1");
  if (prm->s_max < 1) return report_error(SAD_E_INVAL, "s_max must be >= 1");
  const int n = seqs->n, p = prm->p;
  if (n < 2 * p) return report_error(SAD_E_INVAL, "need N >= 2p");
  if (!d_key || !d_bucket || !d_bucket_off || !d_members ||
      (p > 1 && (!d_pivot_key || !d_pivot_id)))
    return report_error(SAD_E_INVAL, "null device array");
  const size_t need = partition_scratch(n, p, nullptr, nullptr);
  if (need > kStaticScratchBytes)
    return report_error(SAD_E_CAPACITY,
                        "partition of " + std::to_string(n) + " ids into " + std::to_string(p) +
                            " buckets needs " + std::to_string(need) +
                            " bytes of scratch; the static scratch holds " +
                            std::to_string(kStaticScratchBytes));
  void* base = nullptr;
  int32_t r = static_scratch(&base);
  if (r) return r;
  PartitionScratch ps{};
  partition_scratch(n, p, static_cast<char*>(base), &ps);
  (void)hipGetLastError();  // start from a clean launch status
  launch_partition_keys(d_key, n, p, ps, d_pivot_key, d_pivot_id, d_bucket, d_bucket_off,
                        d_members, stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return report_error(SAD_E_DEVICE, std::string("partition launch: ") + hipGetErrorString(e));
  return SAD_OK;
}
