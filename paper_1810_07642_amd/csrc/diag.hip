// Term-balance diagnostic of arXiv:1810.07642 (appendix, eq. "magnitude"):
// norms over the lattice, (N^-1 sum_x phi^2)^(1/2), of the terms on the
// right-hand side of the depth-averaged momentum equation (eq. "hydro2"),
// from the current pre-collision state, per component a in {x, y}:
//   pressure_a  = -h d_a p_film
//   friction_a  = -nu alpha_delta(h) u_a
//   viscous_a   = nu lap(h u_a) + 2 nu d_a(div(h u))
//   advection_a = d_x(j_x u_a) + d_y(j_y u_a)
// Derivatives are the isotropic stencil of the step (eq. "derivative"), the
// Laplacian that of eq. "n_laplace"; d_a(div j) applies the derivative
// stencil to the stencil divergence.  Everything is evaluated in FP64.
//
// A workgroup of 16 x 16 lanes handles 16 x 16 output sites at a time: it
// forms h and j on the tile plus a ring of 2 sites in LDS, p and div j on
// the tile plus a ring of 1, then the eight terms on the tile, and
// accumulates their squares; workgroups stride over the tiles and write one
// FP64 partial sum per term, reduced by a second kernel in a fixed order.
#include "device.h"
#include "launch.h"

namespace tflbm {

constexpr int kDT = 16;          // output tile edge
constexpr int kDH = kDT + 4;     // h, j region: tile + ring 2
constexpr int kDP = kDT + 2;     // p, div j region: tile + ring 1

// 3 sum_l w_l c_l phi(x + c_l) on an LDS array of edge E at (i, j) (row i,
// column j): axis weight 1/3, diagonal 1/12.
template <int E>
__device__ __forceinline__ double dx_s(const double (&a)[E][E], int i, int j) {
  return (a[i][j + 1] - a[i][j - 1]) * (1.0 / 3.0) +
         ((a[i + 1][j + 1] - a[i + 1][j - 1]) + (a[i - 1][j + 1] - a[i - 1][j - 1])) * (1.0 / 12.0);
}
template <int E>
__device__ __forceinline__ double dy_s(const double (&a)[E][E], int i, int j) {
  return (a[i + 1][j] - a[i - 1][j]) * (1.0 / 3.0) +
         ((a[i + 1][j + 1] - a[i - 1][j + 1]) + (a[i + 1][j - 1] - a[i - 1][j - 1])) * (1.0 / 12.0);
}
// (1/6) [4 sum_axes + sum_diagonals - 20 phi]
template <int E>
__device__ __forceinline__ double lap_s(const double (&a)[E][E], int i, int j) {
  const double ax = (a[i][j + 1] + a[i][j - 1]) + (a[i + 1][j] + a[i - 1][j]);
  const double dg = (a[i + 1][j + 1] + a[i + 1][j - 1]) + (a[i - 1][j + 1] + a[i - 1][j - 1]);
  return (4.0 * ax + dg - 20.0 * a[i][j]) * (1.0 / 6.0);
}

template <int P, int KF>
__global__ __launch_bounds__(256) void terms_kernel(StepArgs A, double *partial) {
  __shared__ double sh[kDH][kDH], sjx[kDH][kDH], sjy[kDH][kDH];
  __shared__ double sp[kDP][kDP], sdv[kDP][kDP];
  const int tid = threadIdx.y * kDT + threadIdx.x;
  const int nx = A.nx, ny = A.ny;
  const int tx = (nx + kDT - 1) / kDT, ty = (ny + kDT - 1) / kDT;
  const int ntiles = tx * ty;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tx) * kDT, y0 = (tile / tx) * kDT;
    // h and j on the tile plus ring 2 (periodic)
    for (int idx = tid; idx < kDH * kDH; idx += 256) {
      const int i = idx / kDH, j = idx % kDH;
      const int y = wrap(y0 - 2 + i, ny), x = wrap(x0 - 2 + j, nx);
      double d[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) d[l] = (double)pop_at<P>(A.src, l, y, wrap(x - kCx[l], nx), A);
      double dh = d[0];
#pragma unroll
      for (int l = 1; l < 9; ++l) dh += d[l];
      sh[i][j] = A.href + dh;
      sjx[i][j] = ((d[1] - d[5]) + (d[2] - d[6])) + (d[8] - d[4]);
      sjy[i][j] = ((d[3] - d[7]) + (d[2] - d[6])) + (d[4] - d[8]);
    }
    __syncthreads();
    // film pressure and div j on the tile plus ring 1
    for (int idx = tid; idx < kDP * kDP; idx += 256) {
      const int i = idx / kDP + 1, j = idx % kDP + 1;
      const double r = A.hstar / sh[i][j];
      const double phi = ipow(r, A.n_exp) - ipow(r, A.m_exp);
      if constexpr (KF == kGammaKappa) {
        // per-site (-gamma/6, -gamma kappa)
        const int y = wrap(y0 - 2 + i, ny), x = wrap(x0 - 2 + j, nx);
        const auto *pr = (const typename Form<P>::T *)A.kfield + 2 * ((size_t)y * A.ldx + x);
        sp[i - 1][j - 1] = (double)pr[0] * (6.0 * lap_s(sh, i, j)) + (double)pr[1] * phi;
      } else {
        double kap = A.kappa0;
        if constexpr (KF == kKappa) {
          const int y = wrap(y0 - 2 + i, ny), x = wrap(x0 - 2 + j, nx);
          kap = (double)((const typename Form<P>::T *)A.kfield)[(size_t)y * A.ldx + x];
        }
        sp[i - 1][j - 1] = -A.gamma * (lap_s(sh, i, j) + kap * phi);
      }
      sdv[i - 1][j - 1] = dx_s(sjx, i, j) + dy_s(sjy, i, j);
    }
    __syncthreads();
    {
      const int i = threadIdx.y, j = threadIdx.x;  // output site (x0 + j, y0 + i)
      if (x0 + j < nx && y0 + i < ny) {
        const int I = i + 2, J = j + 2;  // in the h, j arrays
        const int Ip = i + 1, Jp = j + 1;  // in the p, div arrays
        const double h = sh[I][J];
        const double ux = sjx[I][J] / h, uy = sjy[I][J] / h;
        const double alpha = 6.0 * h / (2.0 * h * h + 6.0 * A.delta * h + 3.0 * A.delta * A.delta);
        double t[8];
        t[0] = -h * dx_s(sp, Ip, Jp);
        t[1] = -A.nu * alpha * ux;
        t[2] = A.nu * lap_s(sjx, I, J) + 2.0 * A.nu * dx_s(sdv, Ip, Jp);
        t[4] = -h * dy_s(sp, Ip, Jp);
        t[5] = -A.nu * alpha * uy;
        t[6] = A.nu * lap_s(sjy, I, J) + 2.0 * A.nu * dy_s(sdv, Ip, Jp);
        // advection: d_x(j_x u_a) + d_y(j_y u_a) from the ring-1 neighbours
        double q[3][3][4];
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
          for (int b = -1; b <= 1; ++b) {
            const double hh = sh[I + a][J + b], jx = sjx[I + a][J + b], jy = sjy[I + a][J + b];
            const double vx = jx / hh, vy = jy / hh;
            q[a + 1][b + 1][0] = jx * vx;
            q[a + 1][b + 1][1] = jy * vx;
            q[a + 1][b + 1][2] = jx * vy;
            q[a + 1][b + 1][3] = jy * vy;
          }
        auto dxq = [&](int c) {
          return (q[1][2][c] - q[1][0][c]) * (1.0 / 3.0) +
                 ((q[2][2][c] - q[2][0][c]) + (q[0][2][c] - q[0][0][c])) * (1.0 / 12.0);
        };
        auto dyq = [&](int c) {
          return (q[2][1][c] - q[0][1][c]) * (1.0 / 3.0) +
                 ((q[2][2][c] - q[0][2][c]) + (q[2][0][c] - q[0][0][c])) * (1.0 / 12.0);
        };
        t[3] = dxq(0) + dyq(1);
        t[7] = dxq(2) + dyq(3);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += t[c] * t[c];
      }
    }
    __syncthreads();
  }
  // workgroup sums in a fixed order: wave sums, then the four waves
  __shared__ double red[8][4];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    double v = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[c][tid >> 6] = v;
  }
  __syncthreads();
  if (tid < 8) partial[(size_t)tid * gridDim.x + blockIdx.x] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

// out[c] = sqrt(sum_b partial[c][b] / N), one wavefront per term.
__global__ __launch_bounds__(512) void terms_final_kernel(const double *partial, int nb, double inv_n, double *out) {
  const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double v = 0.0;
  for (int b = lane; b < nb; b += 64) v += partial[(size_t)c * nb + b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) out[c] = sqrt(v * inv_n);
}

template <int P>
static void launch_terms_p(const StepArgs &A, int kf, int nb, double *partial, hipStream_t s) {
  const dim3 block(kDT, kDT);
  if (kf == kGammaKappa) terms_kernel<P, kGammaKappa><<<nb, block, 0, s>>>(A, partial);
  else if (kf == kKappa) terms_kernel<P, kKappa><<<nb, block, 0, s>>>(A, partial);
  else terms_kernel<P, kNoField><<<nb, block, 0, s>>>(A, partial);
}

int terms_blocks(int nx, int ny, int max_blocks) {
  const long long ntiles = (long long)((nx + kDT - 1) / kDT) * ((ny + kDT - 1) / kDT);
  return (int)(ntiles < max_blocks ? ntiles : max_blocks);
}

hipError_t launch_terms(int prec, const StepArgs &A, int kf, double *partial, int nb, double *out, hipStream_t s) {
  switch (prec) {
    case kF64: launch_terms_p<kF64>(A, kf, nb, partial, s); break;
    case kF32: launch_terms_p<kF32>(A, kf, nb, partial, s); break;
    default: launch_terms_p<kF16S>(A, kf, nb, partial, s); break;
  }
  terms_final_kernel<<<1, 512, 0, s>>>(partial, nb, 1.0 / ((double)A.nx * (double)A.ny), out);
  return hipGetLastError();
}

}  // namespace tflbm
