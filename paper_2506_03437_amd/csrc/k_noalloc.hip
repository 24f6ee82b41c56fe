// The search entry point that allocates nothing (quake_search_noalloc).
//
// Its search workspace lives in `scratch`, a file-scope device array of
// SCRATCH_BYTES that every device the library runs on holds from module load
// until the process ends.  In host code `scratch` names a host-side stand-in,
// so the array's device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.  All calls on one device share its array and the
// process-wide host counter block below: calls that overlap on one device
// race.  Each call clears what must start at zero with fill kernels.
#include <mutex>

#include "engine.hpp"
#include "index.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = size_t{256} << 20;
constexpr int MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};
int64_t g_host_counters[qk::COUNTERS];

// The current device's copy of `scratch` (looked up on the device's first call).
char* device_scratch() {
  int dev = 0;
  QK_HIP(hipGetDevice(&dev));
  QK_CHECK(dev >= 0 && dev < MAX_DEVICES, QUAKE_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      (void)hipGetLastError();
      throw qk::Error{QUAKE_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc)};
    }
    g_scratch[dev] = p;
  }
  return static_cast<char*>(g_scratch[dev]);
}

}  // namespace

extern "C" int quake_search_noalloc(quake_index* index, const float* q, int64_t nq,
                                    const quake_search_params* params, int64_t* out_ids, float* out_dist,
                                    int32_t* out_nscanned, double* out_recall, void* stream) {
  return qk::run_api([&] {
    char* base = device_scratch();
    qk::search_in_scratch(index, q, nq, params, out_ids, out_dist, out_nscanned, out_recall,
                          reinterpret_cast<hipStream_t>(stream), base, SCRATCH_BYTES, g_host_counters);
  });
}
