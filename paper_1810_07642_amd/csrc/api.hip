// C ABI of the thin-film lattice Boltzmann library: parameter validation,
// workspace layout, launch orchestration and error codes (forward part).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "launch.h"
#include "sim.h"

using namespace tflbm;

namespace tflbm {

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int hip_status(const tflbm_sim *s, hipError_t e) {
  if (e == hipSuccess) return TFLBM_OK;
  if (s) s->last_error = hipGetErrorString(e);
  return TFLBM_EHIP;
}

int choose_rows(int ny, int nstrips, int slots, int min_rows, const char *env_name) {
  if (const char *e = std::getenv(env_name)) {
    const int r = std::atoi(e);
    if (r > 0) return r < ny ? r : ny;
  }
  // As many row chunks as fit in one round of resident wavefronts: a second,
  // partly filled round would leave most of the GPU idle at the end.
  int chunks = slots / (nstrips > 0 ? nstrips : 1);
  if (chunks < 1) chunks = 1;
  int rows = (ny + chunks - 1) / chunks;
  if (rows < min_rows) rows = min_rows;
  if (rows > ny) rows = ny;
  return rows;
}

// Shortest row chunk a tile marches.  On small lattices, where one round of
// tiles cannot fill the GPU anyway, a tile's time is its chain of rows (chunk
// plus halo rows) and short chunks win.  Measured (FP32, microseconds per
// step): the forward step and the one-step reverse pass are fastest with
// one-row chunks wherever the plan picks them (forward 128^2: 5.4 against 9.0
// with four-row chunks; reverse 256^2: 6.4 against 8.7); the two-step reverse
// pass, with ten halo rows per chunk, needs at least four (512^2: 11.3 with
// three rows, 15.1 with two).
constexpr int kMinRowsStep = 1;
constexpr int kMinRowsAdj = 1;
constexpr int kMinRowsAdj2 = 4;
// Three fused steps per pass (omega = 1) are planned once the lattice gives
// every resident slot of the three-step kernel at least this many strip
// rows: below that a tile's sixteen halo rows and longer chain of rows cost
// more than the third of the bytes they save.  Measured (MLUPS, two / three
// steps per pass; strip rows per slot): FP64 768^2 37.4k / 36.0k (6.4),
// 1024^2 43.2k / 46.8k (11.5), 2048^2 51.0k / 64.5k, 4096^2 55.4k / 73.5k;
// FP32 1024^2 69.6k / 66.6k (5.0), 1536^2 92.1k / 106.4k (11.3), 2048^2
// 98.9k / 124.2k, 4096^2 108.1k / 153.1k.  With the general stages the three
// steps' population histories cap a CU at five wavefronts, and two steps per
// pass are as fast or faster (FP64 4096^2 54.8k / 52.7k, FP32 107.2k /
// 108.3k, 2048^2 97.6k / 91.3k).
constexpr int kFuse3MinRowsPerSlot = 8;

// Lattices up to this many sites have steps bound by launch latency and a
// chain of rows, not by bytes: tflbm_step replays blocks of kGraphSteps steps
// from a captured graph there.  Measured per step (FP32 / FP64, plain launches
// against graph replay): 64^2 5.20 / 4.49 against 4.68 / 4.14 us, 128^2 5.29 /
// 4.88 against 4.70 / 4.51, 256^2 6.25 / 6.52 against 5.72 / 6.14, 512^2 9.53
// / 11.07 against 9.20 / 10.99, 1024^2 15.95 / 24.76 against 15.75 / 24.25.
// kGraphSteps is a multiple of four, an even number of buffer swaps whether
// the steps are fused in pairs or not (and with three per pass, 21 + 1
// launches), so a block ends on the parity it started from.
// Capturing and instantiating a block costs about 0.2 ms (3-4 ms for the first
// graph of a process) against 0.03-0.05 ms saved per replayed block at 128^2 to
// 512^2, so a handle captures only once it has run kGraphAfterSteps steps:
// shorter runs (a TFLBMRun forward has a handle of its own) pay nothing.
constexpr int kGraphSteps = 64;
constexpr int64_t kGraphMaxSites = 1 << 20;
constexpr int64_t kGraphAfterSteps = 4 * kGraphSteps;

// Launch shapes of the step kernels for the device current at the call.
void plan_launches(tflbm_sim *s) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int ny = s->p.ny;
  const bool g0 = s->p.g == 0.0;
  int occ1 = step_blocks_per_cu(s->p.prec, s->kfield, 1, g0, s->w1);
  int occ2 = step_blocks_per_cu(s->p.prec, s->kfield, 2, g0, s->w1);
  if (occ1 <= 0) occ1 = 8;
  if (occ2 <= 0) occ2 = 8;
  s->rows = choose_rows(ny, s->nstrips, occ1 * cus, kMinRowsStep, "TFLBM_ROWS");
  s->ntiles = s->nstrips * ((ny + s->rows - 1) / s->rows);
  s->per_xcd = (s->ntiles + 7) / 8;
  // The FP32 fused kernel, bound by its bytes, runs faster with chunks planned
  // for seven resident wavefronts per CU than for the eight its resources
  // allow (taller chunks, fewer halo rows, less contention for HBM); measured
  // MLUPS, eight against seven: 2048^2 97.5k / 101.3k, 3072^2 107.1k / 111.2k,
  // 4096^2 110.3k / 113.5k, 6144^2 118.1k / 118.2k, 8192^2 119.5k / 121.2k,
  // with every chunk count in between slower than both.  FP64 and FP16S are
  // fastest with all eight (FP16S, bound by its VALU, loses 3-7 % with
  // taller chunks).
  const int plan2 = s->p.prec == kF32 && occ2 > 7 ? 7 : occ2;
  s->rows2 = choose_rows(ny, s->nstrips, plan2 * cus, kMinRowsStep, "TFLBM_ROWS2");
  s->ntiles2 = s->nstrips * ((ny + s->rows2 - 1) / s->rows2);
  s->per_xcd2 = (s->ntiles2 + 7) / 8;
  int occ3 = step_blocks_per_cu(s->p.prec, s->kfield, 3, g0, s->w1);
  if (occ3 <= 0) occ3 = 5;
  s->rows3 = choose_rows(ny, s->nstrips, occ3 * cus, kMinRowsStep, "TFLBM_ROWS3");
  s->ntiles3 = s->nstrips * ((ny + s->rows3 - 1) / s->rows3);
  s->per_xcd3 = (s->ntiles3 + 7) / 8;
  // Two fused steps per pass pay off once the one-step plan can no longer give
  // every row a tile of its own in one round of resident wavefronts: below
  // that a tile's time is its chain of rows, 5 for one step against 11 per
  // two fused steps, each of those twice the work.  Measured per step at FP32:
  // 128^2 5.4 vs 6.4 us, 256^2 6.0 vs 6.8, 512^2 9.2 vs 9.4; from 768^2 on
  // the fused pass wins.  FP16S, whose rows take longer to decode, gains from
  // one step per pass up to about 24 one-row tiles per CU (g = 0, per step:
  // 512^2 10.0 vs 12.0 us, 768^2 12.4 vs 14.1; 1024^2 18.5 vs 17.9; with
  // g != 0 likewise 512^2 10.9 vs 12.9, 768^2 13.7 vs 15.1).
  const int64_t one_row_tiles = s->p.prec == kF16S ? 24LL * cus : (int64_t)occ1 * cus;
  s->fuse_fits = (int64_t)s->nstrips * ny > one_row_tiles;
  // Three steps per pass: with the omega = 1 stages, on lattices with long
  // enough chunks (kFuse3MinRowsPerSlot).
  s->fuse3_fits = s->w1 && max_steps_per_pass(s->p.prec, s->w1) >= 3 && s->fuse_fits &&
                  (int64_t)s->nstrips * ny >= kFuse3MinRowsPerSlot * (int64_t)occ3 * cus;
  // FP64 on such lattices: a two-step pass (the remainder of a call whose
  // step count is not a multiple of three) runs the general stages' two-step
  // kernel, which gives the same bits, plans the same chunks (eight
  // wavefronts per CU) and, with its uniform stores, is faster there (4096^2:
  // 570 against 613 us per launch).  Where the two-step pass is the main one
  // (smaller lattices) the omega = 1 kernel stays.
  s->rem2_general = s->fuse3_fits && s->p.prec == kF64;
  // Reverse steps: at most two resident wavefronts per SIMD are planned for
  // (eight per CU).  At 4096^2 FP32 the one-step kernel, which fits three,
  // ran 9% faster with chunks sized for two than for three.
  int aocc1 = adj_blocks_per_cu(s->p.prec, s->kfield == kKappa, 1, s->w1);
  int aocc2 = adj_blocks_per_cu(s->p.prec, s->kfield == kKappa, 2, s->w1);
  aocc1 = aocc1 <= 0 || aocc1 > 8 ? 8 : aocc1;
  aocc2 = aocc2 <= 0 || aocc2 > 8 ? 8 : aocc2;
  s->adj_rows = choose_rows(ny, s->adj_nstrips, aocc1 * cus, kMinRowsAdj, "TFLBM_ADJ_ROWS");
  s->adj_ntiles = s->adj_nstrips * ((ny + s->adj_rows - 1) / s->adj_rows);
  s->adj_per_xcd = (s->adj_ntiles + 7) / 8;
  s->adj2_rows = choose_rows(ny, s->adj_nstrips, aocc2 * cus, kMinRowsAdj2, "TFLBM_ADJ_ROWS2");
  s->adj2_ntiles = s->adj_nstrips * ((ny + s->adj2_rows - 1) / s->adj2_rows);
  s->adj2_per_xcd = (s->adj2_ntiles + 7) / 8;
  // Two reverse steps per pass pay off once the lattice fills the GPU: with
  // fewer tiles of the shortest chunk than resident slots, a tile's time is
  // its chain of rows, which the fused pass makes longer (ten halo rows, two
  // stages per row) than two single passes (four halo rows each).  Measured
  // per step at FP32: single steps win up to 512^2 (10.2 vs 11.2 us), the
  // fused pass from 768^2 on (15.6 vs 20.1; 4096^2: 256 vs 446); at FP64 the
  // two tie at 512^2 (16.9 us) and the fused pass wins from 768^2 on (25.9
  // vs 31.8).
  // With omega = 1 the FP64 one-step pass, which carries three fields per
  // site, runs two wavefronts per SIMD where the two-step pass runs one, and
  // is as fast or faster at every size (per step: 1024^2 33.6 vs 33.3 us,
  // 2048^2 104.0 vs 111.3, 4096^2 393.6 vs 407.4); FP32 keeps two steps per
  // pass (4096^2: 188.8 vs 284.8 us).
  s->adj_fuse_fits = !(s->w1 && s->p.prec == kF64) &&
                     (int64_t)s->adj_nstrips * ((ny + kMinRowsAdj2 - 1) / kMinRowsAdj2) > (int64_t)aocc2 * cus;
  s->graphs = (int64_t)s->p.nx * ny <= kGraphMaxSites;
  if (const char *e = std::getenv("TFLBM_GRAPH")) s->graphs = std::atoi(e) != 0;
}

// Releases the captured step graphs (their kernels name the bound workspace
// and the kernel variant chosen at init); waits for the device first, since a
// replay may still run.
void drop_graphs(tflbm_sim *s) {
  if (!s->gexec[0] && !s->gexec[1]) return;
  (void)hipDeviceSynchronize();
  for (hipGraphExec_t &g : s->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

StepArgs make_step_args(const tflbm_sim *s, int ns) {
  StepArgs A;
  std::memset(&A, 0, sizeof(A));
  A.src = s->ws + (s->cur == 0 ? s->off_a : s->off_b);
  A.dst = s->ws + (s->cur == 0 ? s->off_b : s->off_a);
  A.kfield = s->kfield ? (const void *)(s->ws + s->off_k) : nullptr;
  A.capture = nullptr;
  A.flag = (int *)(s->ws + s->off_flag);
  A.nx = s->p.nx;
  A.ny = s->p.ny;
  A.ldx = s->ldx;
  A.plane = s->plane;
  A.nblk = s->nblk;
  A.nstrips = s->nstrips;
  A.H = ns == 3 ? s->rows3 : ns == 2 ? s->rows2 : s->rows;
  A.ntiles = ns == 3 ? s->ntiles3 : ns == 2 ? s->ntiles2 : s->ntiles;
  A.per_xcd = ns == 3 ? s->per_xcd3 : ns == 2 ? s->per_xcd2 : s->per_xcd;
  A.n_exp = s->p.n_exp;
  A.m_exp = s->p.m_exp;
  A.omega = 1.0 / s->p.tau;
  A.gamma = s->p.gamma;
  A.nu = (s->p.tau - 0.5) / 3.0;
  A.hstar = s->p.hstar;
  A.delta = s->p.delta;
  A.ax = s->p.ax;
  A.ay = s->p.ay;
  A.g = s->p.g;
  A.kappa0 = s->kappa0;
  // the FP32 forms step with href in FP32: take that value everywhere
  A.href = s->p.prec == TFLBM_FP64 ? s->p.href : (double)(float)s->p.href;
  A.qscale = std::ldexp(1.0f, s->p.fp16_scale_log2);
  A.qinv = std::ldexp(1.0f, -s->p.fp16_scale_log2);
  return A;
}

}  // namespace tflbm

extern "C" {

const char *tflbm_version(void) { return "tflbm 0.1 (gfx950)"; }

const char *tflbm_strerror(int code) {
  switch (code) {
    case TFLBM_OK: return "ok";
    case TFLBM_EINVAL: return "invalid argument";
    case TFLBM_EUNSTABLE: return "parameters outside the stable range of the friction recurrence (2 nu/delta^2 >= 2)";
    case TFLBM_EHIP: return "HIP runtime error";
    case TFLBM_ENONFINITE: return "non-finite or non-positive film height";
    case TFLBM_ESTATE: return "call out of order";
    default: return "unknown error";
  }
}

const char *tflbm_last_error(const tflbm_sim *sim) { return sim ? sim->last_error.c_str() : ""; }

void tflbm_default_params(tflbm_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->prec = TFLBM_FP64;
  p->n_exp = 9;
  p->m_exp = 3;
  p->fp16_scale_log2 = 12;
  p->tau = 1.0;
  p->gamma = 0.01;
  p->g = 0.0;
  p->hstar = 0.05;
  p->delta = 1.0;
  p->theta0 = 0.0;
  p->href = 0.0;
}

static bool is_fin(double v) { return std::isfinite(v); }

int tflbm_check_params(const tflbm_params *p) {
  if (!p) return TFLBM_EINVAL;
  if (p->nx < 1 || p->ny < 1) return TFLBM_EINVAL;
  const int64_t ldx = ((int64_t)p->nx + 63) / 64 * 64;
  if ((int64_t)p->ny * ldx >= ((int64_t)1 << 31)) return TFLBM_EINVAL;
  if (p->prec < TFLBM_FP64 || p->prec > TFLBM_FP16S) return TFLBM_EINVAL;
  // one row of records is addressed through a 32-bit buffer range, and every
  // row (population, capture and adjoint records) ends below the offset the
  // kernels' dropped stores aim at (kDropBytes)
  const int64_t nblk = ((int64_t)p->nx + record_sites(p->prec) - 1) / record_sites(p->prec);
  const int64_t astrips = ((int64_t)p->nx + adj_record_columns() - 1) / adj_record_columns();
  if (nblk * record_bytes(p->prec) >= kDropBytes || nblk * capture_record_bytes(p->prec) >= kDropBytes ||
      astrips * adj_record_bytes_max(p->prec) >= kDropBytes)
    return TFLBM_EINVAL;
  if (p->n_exp < 1 || p->n_exp > 32 || p->m_exp < 1 || p->m_exp > 32 || p->n_exp == p->m_exp) return TFLBM_EINVAL;
  if (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24) return TFLBM_EINVAL;
  if (p->gamma_field != 0 && p->gamma_field != 1) return TFLBM_EINVAL;
  if (!is_fin(p->tau) || !(p->tau > 0.5)) return TFLBM_EINVAL;
  if (!is_fin(p->gamma) || p->gamma < 0) return TFLBM_EINVAL;
  if (!is_fin(p->g) || !is_fin(p->ax) || !is_fin(p->ay) || !is_fin(p->theta0)) return TFLBM_EINVAL;
  if (!is_fin(p->hstar) || !(p->hstar > 0)) return TFLBM_EINVAL;
  if (!is_fin(p->delta) || p->delta < 0) return TFLBM_EINVAL;
  if (!is_fin(p->href) || p->href < 0) return TFLBM_EINVAL;
  const double nu = (p->tau - 0.5) / 3.0;
  if (p->delta == 0.0 || 2.0 * nu / (p->delta * p->delta) >= 2.0) return TFLBM_EUNSTABLE;
  return TFLBM_OK;
}

int tflbm_create(const tflbm_params *p, tflbm_sim **out) {
  if (!out) return TFLBM_EINVAL;
  *out = nullptr;
  const int chk = tflbm_check_params(p);
  if (chk == TFLBM_EINVAL) return chk;
  tflbm_sim *s = new (std::nothrow) tflbm_sim();
  if (!s) return TFLBM_EINVAL;
  s->p = *p;
  // omega = 1 exactly: the collision replaces the populations by the
  // equilibrium, and the stages need no population history (TFLBM_OMEGA1=0
  // keeps the general stages, which give the same bits)
  s->w1 = p->tau == 1.0;
  if (const char *e = std::getenv("TFLBM_OMEGA1")) s->w1 = s->w1 && std::atoi(e) != 0;
  s->ldx = (p->nx + 63) / 64 * 64;
  s->plane = (int64_t)p->ny * s->ldx;
  const size_t P = (size_t)s->plane;
  s->nblk = (p->nx + record_sites(p->prec) - 1) / record_sites(p->prec);
  s->pop_bytes = (size_t)p->ny * s->nblk * record_bytes(p->prec);
  s->kf_bytes = (size_t)work_bytes(p->prec) * P * (p->gamma_field ? 2 : 1);  // kappa, or (-gamma/6, -gamma kappa)
  s->n_partials = 1024;
  size_t o = 0;
  s->off_a = o; o = align_up(o + s->pop_bytes, 4096);
  s->off_b = o; o = align_up(o + s->pop_bytes, 4096);
  s->off_k = o; o = align_up(o + s->kf_bytes, 4096);
  s->off_flag = o; o = align_up(o + 256, 256);
  s->off_part = o; o = align_up(o + 8 * 8 * (size_t)s->n_partials, 256);  // up to 8 sums per workgroup
  s->off_out = o; o = align_up(o + 256, 4096);
  s->ws_bytes = o;
  s->kconst = (double)((p->n_exp - 1) * (p->m_exp - 1)) / ((double)(p->n_exp - p->m_exp) * p->hstar);
  s->kappa0 = (1.0 - std::cos(p->theta0)) * s->kconst;
  s->nstrips = s->nblk;  // one marching strip per record column
  if (const char *e = std::getenv("TFLBM_FUSE")) {  // default 0: by lattice size
    const int f = std::atoi(e);
    s->fuse = f <= 1 ? 1 : (f >= 3 ? 3 : 2);
  }
  if (const char *e = std::getenv("TFLBM_ADJ_FUSE")) s->adj_fuse = std::atoi(e) == 1 ? 1 : 2;  // default 0: by lattice size
  s->adj_nstrips = (p->nx + adj_record_columns() - 1) / adj_record_columns();
  *out = s;
  return TFLBM_OK;
}

void tflbm_destroy(tflbm_sim *sim) {
  if (!sim) return;
  drop_graphs(sim);
  if (sim->gstream) (void)hipStreamDestroy(sim->gstream);
  delete sim;
}

size_t tflbm_workspace_bytes(const tflbm_sim *sim) { return sim ? sim->ws_bytes : 0; }

int tflbm_bind(tflbm_sim *sim, void *d_ws, size_t bytes) {
  if (!sim || !d_ws || bytes < sim->ws_bytes || ((uintptr_t)d_ws & 255) != 0) return TFLBM_EINVAL;
  drop_graphs(sim);
  sim->ws = (char *)d_ws;
  sim->initialised = false;
  sim->adj_seeded = false;
  sim->cur = 0;
  sim->steps = 0;
  return TFLBM_OK;
}

int tflbm_init(tflbm_sim *sim, const double *d_h0, const double *d_theta, tflbm_stream_t stream) {
  return tflbm_init_fields(sim, d_h0, d_theta, nullptr, stream);
}

int tflbm_init_fields(tflbm_sim *sim, const double *d_h0, const double *d_theta, const double *d_gamma,
                      tflbm_stream_t stream) {
  if (!sim || !d_h0) return TFLBM_EINVAL;
  if (d_gamma && !sim->p.gamma_field) return TFLBM_EINVAL;
  if (!sim->ws) return TFLBM_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  drop_graphs(sim);
  // set-up of tflbm_mass_noalloc: the address of the static scratch on this device
  double *scr = nullptr;
  int rc = scratch_on_current_device(sim, &scr);
  if (rc) return rc;
  sim->cur = 1;  // init writes into the "dst" of a cur=1 state, i.e. buffer A
  sim->kfield = sim->p.gamma_field ? kGammaKappa : (d_theta != nullptr ? kKappa : kNoField);
  plan_launches(sim);
  StepArgs A = make_step_args(sim);
  rc = hip_status(sim, hipMemsetAsync(sim->ws + sim->off_flag, 0, 256, st));
  if (rc) return rc;
  rc = hip_status(sim, launch_init(sim->p.prec, A, d_h0, d_theta, d_gamma, sim->kfield, sim->kconst, st));
  if (rc) return rc;
  sim->cur = 0;
  sim->steps = 0;
  sim->initialised = true;
  sim->adj_seeded = false;
  return TFLBM_OK;
}

// Launches nsteps steps kernel by kernel: passes of the most fused steps the
// handle allows while that many remain, then shorter ones (with capture: the
// moments of steps i .. i + ns - 1 of a pass, one capture block apart).
// Most steps one launch of tflbm_step fuses on this handle.
static int steps_per_pass(const tflbm_sim *sim) {
  int ns = sim->fuse != 0 ? sim->fuse : (sim->fuse3_fits ? 3 : (sim->fuse_fits ? 2 : 1));
  const int nsmax = max_steps_per_pass(sim->p.prec, sim->w1);
  return ns > nsmax ? nsmax : ns;
}

static int launch_steps(tflbm_sim *sim, int64_t nsteps, void *d_capture, hipStream_t st) {
  const size_t cap_bytes = tflbm_capture_bytes(sim);
  const int ns_max = steps_per_pass(sim);
  int64_t i = 0;
  while (i < nsteps) {
    const int ns = (int)(nsteps - i < ns_max ? nsteps - i : ns_max);
    StepArgs A = make_step_args(sim, ns);
    A.capture = d_capture ? (char *)d_capture + (size_t)i * cap_bytes : nullptr;
    const bool w1 = sim->w1 && !(ns == 2 && !d_capture && sim->rem2_general);
    const int rc = hip_status(sim, launch_step(sim->p.prec, ns, A, sim->kfield, d_capture != nullptr, w1, st));
    if (rc) return rc;
    sim->cur ^= 1;
    sim->steps += ns;
    i += ns;
  }
  return TFLBM_OK;
}

// One block of kGraphSteps steps as a graph launch on `st`; the graph for the
// current parity is captured on first use.  Returns false, with nothing
// launched, where no graph can be used: `st` is itself being captured, or
// capturing failed (graphs are then off for this handle).
static bool graph_block(tflbm_sim *sim, hipStream_t st, int &rc) {
  rc = TFLBM_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t &ex = sim->gexec[sim->cur];
  if (!ex) {
    bool ok = sim->gstream != nullptr || hipStreamCreateWithFlags(&sim->gstream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamBeginCapture(sim->gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const int cur0 = sim->cur;
      const int64_t steps0 = sim->steps;
      const int lrc = launch_steps(sim, kGraphSteps, nullptr, sim->gstream);
      hipGraph_t g = nullptr;
      ok = hipStreamEndCapture(sim->gstream, &g) == hipSuccess && lrc == TFLBM_OK && g != nullptr &&
           sim->cur == cur0 && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
      sim->cur = cur0;  // capturing ran nothing
      sim->steps = steps0;
    }
    if (!ok) {
      ex = nullptr;
      sim->graphs = false;
      (void)hipGetLastError();
      sim->last_error.clear();
      return false;
    }
  }
  rc = hip_status(sim, hipGraphLaunch(ex, st));
  if (rc == TFLBM_OK) sim->steps += kGraphSteps;
  return true;
}

static int run_steps(tflbm_sim *sim, int64_t nsteps, void *d_capture, tflbm_stream_t stream) {
  if (!sim || nsteps < 0) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  int64_t done = 0;
  if (d_capture == nullptr && sim->graphs) {
    while (nsteps - done >= kGraphSteps) {
      if (!sim->gexec[sim->cur] && sim->steps < kGraphAfterSteps) {
        const int rc = launch_steps(sim, kGraphSteps, nullptr, st);
        if (rc) return rc;
      } else {
        int rc = TFLBM_OK;
        if (!graph_block(sim, st, rc)) break;
        if (rc) return rc;
      }
      done += kGraphSteps;
    }
  }
  return launch_steps(sim, nsteps - done, d_capture, st);
}

int tflbm_step(tflbm_sim *sim, int64_t nsteps, tflbm_stream_t stream) {
  return run_steps(sim, nsteps, nullptr, stream);
}

int tflbm_step_capture(tflbm_sim *sim, int64_t nsteps, void *d_capture, tflbm_stream_t stream) {
  if (!d_capture) return TFLBM_EINVAL;
  return run_steps(sim, nsteps, d_capture, stream);
}

int64_t tflbm_step_count(const tflbm_sim *sim) { return sim ? sim->steps : -1; }

int tflbm_steps_per_pass(const tflbm_sim *sim) {
  if (!sim) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  return steps_per_pass(sim);
}

int tflbm_step_graphs(const tflbm_sim *sim) {
  return sim ? (sim->gexec[0] != nullptr) + (sim->gexec[1] != nullptr) : -1;
}

int tflbm_read(const tflbm_sim *sim, double *d_h, double *d_ux, double *d_uy, tflbm_stream_t stream) {
  if (!sim) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  if (!d_h && !d_ux && !d_uy) return TFLBM_OK;
  StepArgs A = make_step_args(sim);
  return hip_status(sim, launch_read(sim->p.prec, A, d_h, d_ux, d_uy, (hipStream_t)stream));
}

int tflbm_mass(const tflbm_sim *sim, double *h_mass, tflbm_stream_t stream) {
  if (!sim || !h_mass) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  StepArgs A = make_step_args(sim);
  int rc = hip_status(sim, launch_mass(sim->p.prec, A, (double *)(sim->ws + sim->off_part), sim->n_partials,
                                       (double *)(sim->ws + sim->off_out), st));
  if (rc) return rc;
  rc = hip_status(sim, hipMemcpyAsync(h_mass, sim->ws + sim->off_out, sizeof(double), hipMemcpyDeviceToHost, st));
  if (rc) return rc;
  return hip_status(sim, hipStreamSynchronize(st));
}

int tflbm_term_norms(const tflbm_sim *sim, double *h_norms, tflbm_stream_t stream) {
  if (!sim || !h_norms) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  StepArgs A = make_step_args(sim);
  const int nb = terms_blocks(sim->p.nx, sim->p.ny, sim->n_partials);
  int rc = hip_status(sim, launch_terms(sim->p.prec, A, sim->kfield, (double *)(sim->ws + sim->off_part), nb,
                                        (double *)(sim->ws + sim->off_out), st));
  if (rc) return rc;
  rc = hip_status(sim, hipMemcpyAsync(h_norms, sim->ws + sim->off_out, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  if (rc) return rc;
  return hip_status(sim, hipStreamSynchronize(st));
}

int tflbm_check(const tflbm_sim *sim, tflbm_stream_t stream) {
  if (!sim) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  int flag = 0;
  int rc = hip_status(sim, hipMemcpyAsync(&flag, sim->ws + sim->off_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  if (rc) return rc;
  rc = hip_status(sim, hipStreamSynchronize(st));
  if (rc) return rc;
  return flag ? TFLBM_ENONFINITE : TFLBM_OK;
}

size_t tflbm_state_bytes(const tflbm_sim *sim) { return sim ? sim->pop_bytes : 0; }

// A population buffer is whole 128-byte lines; the record-copy kernel moves it
// when both ends are 16-byte aligned (the workspace always is), the runtime's
// copy otherwise.
static hipError_t copy_state(const void *src, void *dst, size_t bytes, hipStream_t st) {
  if (((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0 && bytes % 16 == 0)
    return launch_copy(src, dst, bytes, st);
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
}

int tflbm_state_save(const tflbm_sim *sim, void *d_dst, tflbm_stream_t stream) {
  if (!sim || !d_dst) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  const char *src = sim->ws + (sim->cur == 0 ? sim->off_a : sim->off_b);
  return hip_status(sim, copy_state(src, d_dst, sim->pop_bytes, (hipStream_t)stream));
}

int tflbm_state_load(tflbm_sim *sim, const void *d_src, int64_t step, tflbm_stream_t stream) {
  if (!sim || !d_src || step < 0) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  char *dst = sim->ws + (sim->cur == 0 ? sim->off_a : sim->off_b);
  const int rc = hip_status(sim, copy_state(d_src, dst, sim->pop_bytes, (hipStream_t)stream));
  if (rc) return rc;
  sim->steps = step;
  return TFLBM_OK;
}

size_t tflbm_capture_bytes(const tflbm_sim *sim) {
  return sim ? (size_t)sim->p.ny * sim->nblk * capture_record_bytes(sim->p.prec) : 0;
}

}  // extern "C"
