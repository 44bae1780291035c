// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace tflbm {

// The buffer offset at which the kernels aim the stores they drop (halo lanes
// and rows without output: the buffer range check discards them).  Every row
// of every buffer (population, capture and adjoint records) must end below it,
// which tflbm_check_params enforces.
constexpr int kDropBytes = 0x7fff0000;

// Sites per population record (= output columns of one marching strip) and
// bytes per record, for a storage form.
int record_sites(int prec);
int capture_record_bytes(int prec);
// Workgroups of the term-balance diagnostic and its launcher (partial: 8 x nb doubles).
int terms_blocks(int nx, int ny, int max_blocks);
hipError_t launch_terms(int prec, const StepArgs &A, int kfield, double *partial, int nb, double *out, hipStream_t s);
int record_bytes(int prec);

// ns fused time steps in one pass (1, 2 or 3; src at time t, dst at time
// t + ns).  kfield: the per-site field the step reads: 0 none, 1 kappa, 2 the
// pairs (-gamma/6, -gamma kappa) of a position-dependent surface tension.
// w1: omega = 1 (tau = 1), the stages without a population history.
hipError_t launch_step(int prec, int ns, const StepArgs &A, int kfield, bool capture, bool w1, hipStream_t s);
// Most fused steps per pass of a storage form: its halo columns allow three
// per step, and three need the omega = 1 stages.
int max_steps_per_pass(int prec, bool w1);
// Resident one-wavefront workgroups per CU of the step kernel (0 if unknown).
int step_blocks_per_cu(int prec, int kfield, int ns, bool g0, bool w1);
hipError_t launch_init(int prec, const StepArgs &A, const double *h0, const double *theta, const double *gamma,
                       int field, double kconst, hipStream_t s);
hipError_t launch_read(int prec, const StepArgs &A, double *h, double *ux, double *uy, hipStream_t s);
hipError_t launch_mass(int prec, const StepArgs &A, double *partial, int np, double *out, hipStream_t s);
// Device-to-device copy of `bytes` (a multiple of 16; both pointers 16-byte
// aligned) by the library's record-copy kernel.
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// Reverse-mode kernels.
struct AdjArgs;
// w1: omega = 1, the adjoint carried between steps as three fields per site.
hipError_t launch_adj_seed(int prec, const AdjArgs &B, const double *grad_h, bool w1, hipStream_t s);
hipError_t launch_adj_step(int prec, const AdjArgs &B, bool kfield, int ns, bool w1, hipStream_t s);
hipError_t launch_adj_finish(int prec, const AdjArgs &B, const double *h0, const double *theta, double theta0,
                             double kconst, double *grad_h0, double *grad_theta, bool w1, hipStream_t s);
int adj_record_columns();
// Bytes per strip of the largest adjoint row (records of either kind, or
// the dLoss/dkappa records) for a storage form.
int adj_record_bytes_max(int prec);
int adj_blocks_per_cu(int prec, bool kfield, int ns, bool w1);

}  // namespace tflbm
