// Host-side state behind the opaque tflbm_sim handle (internal).
#pragma once

#include <string>

#include "../../include/tflbm.h"
#include "device.h"

struct tflbm_sim {
  tflbm_params p;
  int ldx = 0;            // row pitch in elements (nx rounded up to 64)
  int64_t plane = 0;      // ny * ldx
  int nblk = 0;           // population records per row
  size_t pop_bytes = 0;   // one population buffer
  size_t kf_bytes = 0;    // kappa field
  size_t off_a = 0, off_b = 0, off_k = 0, off_flag = 0, off_part = 0, off_out = 0, ws_bytes = 0;
  int n_partials = 0;
  char *ws = nullptr;     // bound device workspace
  bool initialised = false;
  int kfield = 0;         // FieldKind: kappa (theta field given at init) or the gamma-kappa pairs read per site
  int cur = 0;            // 0: buffer A holds the current populations
  int64_t steps = 0;
  double kconst = 0.0;    // (n - 1)(m - 1)/((n - m) h_*)
  double kappa0 = 0.0;    // kappa of the uniform theta0
  // launch shapes of the forward step: one, two and three fused steps per pass
  int nstrips = 0, rows = 0, ntiles = 0, per_xcd = 0;
  int rows2 = 0, ntiles2 = 0, per_xcd2 = 0;
  int rows3 = 0, ntiles3 = 0, per_xcd3 = 0;
  int fuse = 0;           // most steps per pass: 1, 2 or 3; 0 = by lattice size (fuse3_fits, fuse_fits)
  bool fuse_fits = false; // the lattice is too large for one round of one-row tiles
  bool fuse3_fits = false;  // three steps per pass (omega = 1) beat two on this lattice
  bool rem2_general = false;  // FP64, omega = 1, three steps per pass: two-step passes run the general stages
  bool w1 = false;        // omega = 1 (tau = 1): the stages without a population history
  // launch-bound lattices: blocks of steps replayed from captured graphs, one
  // per starting buffer parity, captured on a stream of the library's own
  bool graphs = false;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // reverse pass
  int adj_cur = 0;        // 0: first adjoint buffer holds the current adjoint
  bool adj_seeded = false;
  int adj_nstrips = 0;    // strips of the adjoint records (both reverse kernels march them)
  int adj_rows = 0, adj_ntiles = 0, adj_per_xcd = 0;      // one step per pass
  int adj2_rows = 0, adj2_ntiles = 0, adj2_per_xcd = 0;   // two steps per pass
  int adj_fuse = 0;       // reverse steps per pass: 1, 2 (when possible), 0 = 2 if adj_fuse_fits
  bool adj_fuse_fits = false;  // the lattice fills the GPU with two-step tiles
  mutable std::string last_error;
};

namespace tflbm {

// Bytes per element of the working type.
inline int work_bytes(int prec) { return prec == kF64 ? 8 : 4; }

// StepArgs for the current state of `s` (src = current, dst = other buffer),
// shaped for `ns` fused steps per pass.
StepArgs make_step_args(const tflbm_sim *s, int ns = 1);

// Records a HIP error on the handle and returns TFLBM_EHIP (or TFLBM_OK).
int hip_status(const tflbm_sim *s, hipError_t e);

// Rows per chunk of a marching launch with `nstrips` strips over ny rows, given
// `slots` resident wavefronts; an environment variable may override it.
int choose_rows(int ny, int nstrips, int slots, int min_rows, const char *env_name);

// Chooses the launch shapes of the step kernels (needs the device).
void plan_launches(tflbm_sim *s);

// Releases the captured step graphs of `s`, after waiting for the device.
void drop_graphs(tflbm_sim *s);

// Device address of the library's static reduction scratch on the current
// device (tflbm_mass_noalloc), looked up once per device.
int scratch_on_current_device(const tflbm_sim *s, double **out);

}  // namespace tflbm
