// Allocation-free entry point: the total-mass reduction with its partial sums
// in a static device array of the library instead of the handle's workspace,
// and its result left in device memory, so that a caller that cannot allocate
// or synchronise (code under graph capture, serving loops) can still call it.
#include <mutex>

#include "launch.h"
#include "sim.h"

namespace tflbm {

// Partial sums of the two-pass mass reduction (one per workgroup of the first
// pass).  Each GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: kernels receive the address looked up by scratch_on_current_device.
constexpr int kScratchPartials = 1024;
static __device__ __align__(256) double scratch[kScratchPartials];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_on_current_device(const tflbm_sim *s, double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(s, e);
  if (dev < 0 || dev >= kMaxDevices) {
    if (s) s->last_error = "device index beyond the library's table of scratch arrays";
    return TFLBM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return hip_status(s, e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return TFLBM_OK;
}

}  // namespace tflbm

using namespace tflbm;

extern "C" int tflbm_mass_noalloc(const tflbm_sim *sim, double *d_mass, tflbm_stream_t stream) {
  if (!sim || !d_mass) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  if (sim->n_partials < 1 || sim->n_partials > kScratchPartials) {
    sim->last_error = "the mass reduction needs more partial sums than the static scratch array holds (1024)";
    return TFLBM_EINVAL;
  }
  double *partial = nullptr;
  const int rc = scratch_on_current_device(sim, &partial);
  if (rc) return rc;
  const StepArgs A = make_step_args(sim);
  // every partial the final pass reads is written by the first pass: nothing to clear
  return hip_status(sim, launch_mass(sim->p.prec, A, partial, sim->n_partials, d_mass, (hipStream_t)stream));
}
