// Forward kernels of the thin-film lattice Boltzmann method (arXiv:1810.07642,
// Sec. II) other than the step: initial populations, readout of h and u, the
// FP64 mass reduction and the record copy; and the dispatch of the step
// kernels (step.h) to the translation units of the storage forms and stages.
#include "step.h"

namespace tflbm {

extern template hipError_t launch_step_form<kF64, false>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF64, false>(int, int, bool);
extern template hipError_t launch_step_form<kF64, true>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF64, true>(int, int, bool);
extern template hipError_t launch_step_form<kF32, false>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF32, false>(int, int, bool);
extern template hipError_t launch_step_form<kF32, true>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF32, true>(int, int, bool);
extern template hipError_t launch_step_form<kF16S, false>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF16S, false>(int, int, bool);
extern template hipError_t launch_step_form<kF16S, true>(int, const StepArgs &, int, bool, hipStream_t);
extern template int step_occupancy_form<kF16S, true>(int, int, bool);

// ---- initial populations and kappa ------------------------------------------
// f_l = f_l^eq(h0, u = 0): h0 - 5 g h0^2/6 (rest), g h0^2/6 (axes), g h0^2/24
// (diagonals), stored as d_l = f_l - E_l(href), i.e. with dh = h0 - href and
// q = g dh (h0 + href): dh - 5 q/6, q/6, q/24; kappa = (1 - cos theta)(n - 1)
// (m - 1)/((n - m) h_*) (Sec. II).
template <int P> __device__ __forceinline__ char *pop_ptr(char *buf, int l, int y, int c, const StepArgs &A) {
  constexpr int B = Form<P>::B;
  const int blk = c / B, pos = c - blk * B;
  char *rec = buf + ((size_t)y * A.nblk + blk) * Form<P>::RB + seg_offset<P>(l);
  const int es = (P == kF64) ? 8 : ((P == kF16S && l != 0) ? 2 : 4);
  return rec + (size_t)pos * es;
}

template <int P>
__global__ void init_kernel(StepArgs A, const double *h0, const double *theta, const double *gamma, int field,
                            double kconst) {
  using T = typename Form<P>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const double h = h0[(size_t)y * A.nx + x];
  if (!(h > 0.0 && h < INFINITY)) atomicOr(A.flag, 1);
  const double dh = h - A.href;
  const double q = A.g * dh * (h + A.href);
  double e[9];
  e[0] = dh - q * (5.0 / 6.0);
  for (int l = 1; l < 9; ++l) e[l] = (l & 1) ? q * (1.0 / 6.0) : q * (1.0 / 24.0);
  if constexpr (P == kF64 || P == kF32) {
    for (int l = 0; l < 9; ++l) *(T *)pop_ptr<P>(A.dst, l, y, wrap(x - kCx[l], A.nx), A) = (T)e[l];
  } else {
    // FP16S: the state is written as if emitted by a step: site (xs, ys)'s s
    // is the sum of the deviations it "emitted", its rest population and the
    // moving ones that sit at its neighbours (e_l of their h0), and each
    // moving population is stored as its FP16 difference from the rest
    // equilibrium of its source site.
    auto eq_dev = [&](int xs, int ys, int l) {
      const double hh = h0[(size_t)wrap(ys, A.ny) * A.nx + wrap(xs, A.nx)];
      const double dd = hh - A.href, qq = A.g * dd * (hh + A.href);
      return l == 0 ? dd - qq * (5.0 / 6.0) : ((l & 1) ? qq * (1.0 / 6.0) : qq * (1.0 / 24.0));
    };
    auto s_of = [&](int xs, int ys) {
      double sum = eq_dev(xs, ys, 0);
      for (int m = 1; m < 9; ++m) sum += eq_dev(xs + kCx[m], ys + kCy[m], m);
      return (float)sum;
    };
    const float g16 = (float)A.g, h2 = 2.0f * (float)A.href;
    *(float *)pop_ptr<P>(A.dst, 0, y, x, A) = s_of(x, y);
    for (int l = 1; l < 9; ++l) {
      const Rest16 es = rest16(s_of(x - kCx[l], y - kCy[l]), g16, h2);
      const __half dq = __float2half_rn(((float)e[l] - rest16_l(es, l)) * A.qscale);
      *(__half *)pop_ptr<P>(A.dst, l, y, wrap(x - kCx[l], A.nx), A) = dq;
    }
  }
  if (field == kKappa) {
    const double th = theta[(size_t)y * A.nx + x];
    ((T *)A.kfield)[(size_t)y * A.ldx + x] = (T)((1.0 - cos(th)) * kconst);
  } else if (field == kGammaKappa) {
    // (a, b) = (-gamma/6, -gamma kappa), each rounded to T as the scalar path
    // rounds its constants (-gamma/6) and (-gamma) and the product of (-gamma)
    // with kappa in T: a uniform field steps bit for bit like the scalar path
    const double gm = gamma != nullptr ? gamma[(size_t)y * A.nx + x] : A.gamma;
    if (!(gm >= 0.0 && gm < INFINITY)) atomicOr(A.flag, 1);
    const T kap = theta != nullptr ? (T)((1.0 - cos(theta[(size_t)y * A.nx + x])) * kconst) : (T)A.kappa0;
    T *pr = (T *)A.kfield + 2 * ((size_t)y * A.ldx + x);
    pr[0] = (T)(-gm / 6.0);
    pr[1] = (T)(-gm) * kap;
  }
}

// ---- readout: h = href + sum d and u = j/h in FP64 from the stored deviations --
template <int P>
__global__ void read_kernel(StepArgs A, double *hout, double *uxo, double *uyo) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  double f[9];
  for (int l = 0; l < 9; ++l) f[l] = (double)pop_at<P>(A.src, l, y, wrap(x - kCx[l], A.nx), A);
  double dh = f[0];
  for (int l = 1; l < 9; ++l) dh += f[l];
  const double h = A.href + dh;
  const double jx = f[1] + f[2] - f[4] - f[5] - f[6] + f[8];
  const double jy = f[2] + f[3] + f[4] - f[6] - f[7] - f[8];
  const size_t od = (size_t)y * A.nx + x;
  if (hout) hout[od] = h;
  if (uxo) uxo[od] = jx / h;
  if (uyo) uyo[od] = jy / h;
}

// ---- mass: deterministic two-pass FP64 reduction ------------------------------
// sum over sites of sum_l d_l, plus nx ny href.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int P>
__global__ __launch_bounds__(256) void mass_partial_kernel(StepArgs A, double *partial) {
  __shared__ double red[4];
  const int64_t n = (int64_t)A.nx * A.ny;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / A.nx), c = (int)(i % A.nx);
    if constexpr (P == kF16S) {
      acc += (double)src16_at(A.src, y, c, A);  // a site's nine deviations add up to its s
    } else {
      double s = 0.0;
      for (int l = 0; l < 9; ++l) s += (double)pop_at<P>(A.src, l, y, c, A);
      acc += s;
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void mass_final_kernel(const double *partial, int np, double base, double *out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = base + ((red[0] + red[1]) + (red[2] + red[3]));
}

// ---- record copy: checkpoints, and the bandwidth ceiling of one pass ------------
// Copies n16 16-byte words (a population buffer is whole 128-byte lines).
// Workgroup b copies the range [b per_block, (b + 1) per_block); each lane
// has four 16-byte loads in flight before its stores.  Loads and
// stores are non-temporal: nothing reads the copied bytes again soon.  A pass
// of the step reads and writes every record once plus its halo re-reads, so
// this copy's rate is the most that pass could reach on this GPU.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                   int64_t n16, int64_t per_block) {
  const int64_t begin = (int64_t)blockIdx.x * per_block;
  const int64_t end = begin + per_block < n16 ? begin + per_block : n16;
  for (int64_t i = begin + threadIdx.x; i < end; i += 4 * 256) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * 256 < end) v[u] = __builtin_nontemporal_load(src + i + u * 256);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * 256 < end) __builtin_nontemporal_store(v[u], dst + i + u * 256);
  }
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  // one 16 KB chunk per workgroup: consecutive workgroups stream adjacent
  // chunks, so the chunks in flight form one moving window over the buffer.
  // Measured on a 1.24 GB buffer: 6.3 TB/s, against 5.3 TB/s for 4096
  // workgroups each streaming a contiguous 300 KB range.
  constexpr int64_t kPer = 4 * 256;  // 16-byte words per workgroup
  const int64_t nb = (n16 + kPer - 1) / kPer;
  copy_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>((const u32x4 *)src, (u32x4 *)dst, n16, kPer);
  return hipGetLastError();
}

hipError_t launch_step(int prec, int ns, const StepArgs &A, int kf, bool cap, bool w1, hipStream_t s) {
  if (ns < 1 || ns > max_steps_per_pass(prec, w1)) return hipErrorInvalidValue;
  switch (prec) {
    case kF64: return w1 ? launch_step_form<kF64, true>(ns, A, kf, cap, s) : launch_step_form<kF64, false>(ns, A, kf, cap, s);
    case kF32: return w1 ? launch_step_form<kF32, true>(ns, A, kf, cap, s) : launch_step_form<kF32, false>(ns, A, kf, cap, s);
    default: return w1 ? launch_step_form<kF16S, true>(ns, A, kf, cap, s) : launch_step_form<kF16S, false>(ns, A, kf, cap, s);
  }
}

int max_steps_per_pass(int prec, bool) {
  return prec == kF64 ? Form<kF64>::NSMAX : (prec == kF32 ? Form<kF32>::NSMAX : Form<kF16S>::NSMAX);
}

int step_blocks_per_cu(int prec, int kf, int ns, bool g0, bool w1) {
  switch (prec) {
    case kF64: return w1 ? step_occupancy_form<kF64, true>(kf, ns, g0) : step_occupancy_form<kF64, false>(kf, ns, g0);
    case kF32: return w1 ? step_occupancy_form<kF32, true>(kf, ns, g0) : step_occupancy_form<kF32, false>(kf, ns, g0);
    default: return w1 ? step_occupancy_form<kF16S, true>(kf, ns, g0) : step_occupancy_form<kF16S, false>(kf, ns, g0);
  }
}

int record_sites(int prec) { return prec == kF64 ? Form<kF64>::B : (prec == kF32 ? Form<kF32>::B : Form<kF16S>::B); }
int capture_record_bytes(int prec) {
  return prec == kF64 ? cap_record_bytes<kF64>() : (prec == kF32 ? cap_record_bytes<kF32>() : cap_record_bytes<kF16S>());
}
int record_bytes(int prec) {
  return prec == kF64 ? Form<kF64>::RB : (prec == kF32 ? Form<kF32>::RB : Form<kF16S>::RB);
}

hipError_t launch_init(int prec, const StepArgs &A, const double *h0, const double *theta, const double *gamma,
                       int field, double kconst, hipStream_t s) {
  const dim3 block(256), grid((A.nx + 255) / 256, A.ny);
  switch (prec) {
    case kF64: init_kernel<kF64><<<grid, block, 0, s>>>(A, h0, theta, gamma, field, kconst); break;
    case kF32: init_kernel<kF32><<<grid, block, 0, s>>>(A, h0, theta, gamma, field, kconst); break;
    default: init_kernel<kF16S><<<grid, block, 0, s>>>(A, h0, theta, gamma, field, kconst); break;
  }
  return hipGetLastError();
}

hipError_t launch_read(int prec, const StepArgs &A, double *h, double *ux, double *uy, hipStream_t s) {
  const dim3 block(256), grid((A.nx + 255) / 256, A.ny);
  switch (prec) {
    case kF64: read_kernel<kF64><<<grid, block, 0, s>>>(A, h, ux, uy); break;
    case kF32: read_kernel<kF32><<<grid, block, 0, s>>>(A, h, ux, uy); break;
    default: read_kernel<kF16S><<<grid, block, 0, s>>>(A, h, ux, uy); break;
  }
  return hipGetLastError();
}

hipError_t launch_mass(int prec, const StepArgs &A, double *partial, int np, double *out, hipStream_t s) {
  switch (prec) {
    case kF64: mass_partial_kernel<kF64><<<np, 256, 0, s>>>(A, partial); break;
    case kF32: mass_partial_kernel<kF32><<<np, 256, 0, s>>>(A, partial); break;
    default: mass_partial_kernel<kF16S><<<np, 256, 0, s>>>(A, partial); break;
  }
  mass_final_kernel<<<1, 256, 0, s>>>(partial, np, (double)A.nx * (double)A.ny * A.href, out);
  return hipGetLastError();
}

}  // namespace tflbm
