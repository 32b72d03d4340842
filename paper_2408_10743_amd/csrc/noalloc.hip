// noalloc.hip -- qd_round_min_noalloc: one enumeration round for callers that
// cannot allocate device memory.  It runs the same host plan and kernels as
// qd_round_min on an arena executor whose device memory is one fixed array
// per GPU, and allocates nothing from the driver.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/qdist.h"
#include "engine.hpp"

namespace {

// All device memory of qd_round_min_noalloc on one GPU: element rows, e_r
// tables, saved and tops tables, tile plans, the code's state, counters and
// witness slots, carved in order by the arena executor on every call.  Each
// GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, never a device address:
// host code uses the address looked up by device_scratch instead.
static __device__ __align__(256) unsigned char scratch[QD_NOALLOC_SCRATCH_BYTES];

struct DeviceScratch {
  void *ptr = nullptr;  // device address of this GPU's `scratch`
  std::mutex mu;        // calls on one GPU run one at a time
};

// This GPU's scratch address, looked up once per device with that device
// current (after checking that it is a gfx950).
int device_scratch(DeviceScratch **out) {
  static std::mutex mu;
  static std::vector<std::unique_ptr<DeviceScratch>> per_dev;
  int dev = 0, cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0 || hipGetDevice(&dev) != hipSuccess) return QD_ERR_DEVICE;
  std::lock_guard<std::mutex> g(mu);
  if (int(per_dev.size()) <= dev) per_dev.resize(size_t(dev) + 1);
  if (!per_dev[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess || !std::strstr(prop.gcnArchName, "gfx950"))
      return QD_ERR_DEVICE;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QD_ERR_DEVICE;
    per_dev[dev] = std::make_unique<DeviceScratch>();
    per_dev[dev]->ptr = p;
  }
  *out = per_dev[dev].get();
  return QD_OK;
}

}  // namespace

int qd_round_min_noalloc(const uint8_t *rows, const int *dims, int P, int n, int t, int *wmin, uint8_t *witness,
                         unsigned long long *count, int partial_words, void *stream) {
  DeviceScratch *ds = nullptr;
  int rc = device_scratch(&ds);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ds->mu);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int out = QD_ERR_DEVICE;
  {
    qd::Executor ex(s, ds->ptr, QD_NOALLOC_SCRATCH_BYTES);
    if (ex.ok())
      out = qd::one_round(rows, dims, P, n, t, partial_words, 0, wmin, witness, count, nullptr, 0, nullptr, &ex);
  }
  // No kernel of this call may still use the scratch when the next starts.
  if (hipStreamSynchronize(s) != hipSuccess && out == QD_OK) out = QD_ERR_DEVICE;
  return out;
}
