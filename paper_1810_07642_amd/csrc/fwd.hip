// Forward kernels of the thin-film lattice Boltzmann method (arXiv:1810.07642,
// Sec. II): initial populations, the fused time step, readout of h and u, and
// the FP64 mass reduction.
//
// Layout (HBM): populations are structure-of-arrays planes [9][ny][ldx]
// (x fastest, ldx = nx rounded up to 64) in "push" form: plane l holds the
// pre-collision f_l(x) at x itself, so all nine populations of a site are
// read from the site's own address.  Two such buffers ping-pong.
//
// Fused step: one wavefront owns a strip of 64*V - 4 output columns (V
// columns per lane, plus two halo columns on each side) and a chunk of H
// rows, and marches down the rows.  For every new row it reads the nine
// planes once (coalesced), forms h; one row later the film pressure of the
// previous row (Laplacian of h and disjoining term); one more row later the
// isotropic pressure gradient, the forces, the equilibrium and the collision
// of the row two above, whose post-collision populations are written to
// their streaming destinations x + c_l.  The stencil neighbours in x come
// from adjacent lanes (cross-lane shuffles); the three-row windows of h and
// p stay in registers.  No LDS, no barriers.  The only redundant HBM/L2
// reads are the 4 halo columns per strip and the 4 halo rows per chunk.
#include <type_traits>

#include "device.h"
#include "launch.h"

namespace tflbm {

// Aligned store of one population row for the two-column lanes (V = 2).
// `val` holds the post-collision values of the lane's own columns (a, a+1);
// the destination of column c is c + cx.  Each lane writes the aligned pair
// (col0, col0 + 1) of the destination row, taking the value of the column to
// its left (cx = +1) or right (cx = -1) from the neighbouring lane, and only
// the elements whose source column belongs to this strip.  `ok0`/`ok1` tell
// whether the sources of the two destination elements are in the strip.
template <typename E>
__device__ __forceinline__ void store_pair(E *row, int col0, E v0, E v1, bool ok0, bool ok1) {
  if (ok0 && ok1) {
    if constexpr (sizeof(E) == 4) *(float2 *)(row + col0) = make_float2(v0, v1);
    else *(__half2 *)(row + col0) = __halves2half2(v0, v1);
  } else {
    if (ok0) row[col0] = v0;
    if (ok1) row[col0 + 1] = v1;
  }
}

__device__ __forceinline__ __half half_from_left(__half v) {
  return __ushort_as_half((unsigned short)__shfl_up((int)__half_as_ushort(v), 1));
}
__device__ __forceinline__ __half half_from_right(__half v) {
  return __ushort_as_half((unsigned short)__shfl_down((int)__half_as_ushort(v), 1));
}

template <int P, bool KF, bool CAP>
__global__ __launch_bounds__(64) void step_kernel(StepArgs A) {
  using T = typename Form<P>::T;
  constexpr int V = Form<P>::V;
  constexpr int OUTW = 64 * V - 4;
  // populations of rows r-1 and r-2, each lane's own columns
  __shared__ T hist[2][9][64 * V];

  // XCD-aware tile order: consecutive workgroups land on different XCDs
  // (round robin), so give each XCD a contiguous block of tiles.
  const int b = blockIdx.x;
  const int tile = (b & 7) * A.per_xcd + (b >> 3);
  if (tile >= A.ntiles) return;
  const int strip = tile % A.nstrips;
  const int chunk = tile / A.nstrips;
  const int x0 = strip * OUTW;
  const int y0 = chunk * A.H;
  const int yend = min(y0 + A.H, A.ny);
  const int xend = min(x0 + OUTW, A.nx);
  const int lane = threadIdx.x;
  const int nx = A.nx, ny = A.ny, ldx = A.ldx;

  const int a = x0 - 2 + V * lane;  // first (unwrapped) column of this lane
  int col[V], colE[V], colW[V];
  bool out[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    col[v] = wrap(a + v, nx);
    colE[v] = wrap(a + v + 1, nx);
    colW[v] = wrap(a + v - 1, nx);
    out[v] = (a + v >= x0) && (a + v < xend);
  }
  bool vec = true;
  if constexpr (V == 2) vec = ((col[0] & 1) == 0) && (col[1] == col[0] + 1);
  // aligned pair stores need every lane of the wave on an aligned pair
  const bool pairs = (V == 2) && __all(vec);
  // sources of the aligned destination pair for cx = +1 and cx = -1
  const bool srcE0 = (a - 1 >= x0) && (a - 1 < xend);  // column a-1 (cx = +1, element 0)
  const bool srcW1 = (a + 2 >= x0) && (a + 2 < xend);  // column a+2 (cx = -1, element 1)

  const T omega = (T)A.omega, gamma = (T)A.gamma, nu = (T)A.nu, hstar = (T)A.hstar;
  const T ax = (T)A.ax, ay = (T)A.ay, g = (T)A.g;
  const T kap0 = (T)A.kappa0;
  const T cA = (T)(3.0 * kW[1]), cD = (T)(3.0 * kW[2]);  // gradient stencil weights
  const T three_delta2 = (T)(3.0 * A.delta * A.delta), six_delta = (T)(6.0 * A.delta);
  const int n_exp = A.n_exp, m_exp = A.m_exp;

  T fa[9][V], fb[9][V];  // rows in flight: r (being consumed) and r+1
  T h0[V + 2], h1[V + 2], h2[V + 2];
  T p1[V + 2], p2[V + 2], p3[V + 2];
  T kn[V], kr[V];
  int bad = 0;

  const int K = (yend - y0) + 4;
  int ry = wrap(y0 - 2, ny);          // row r
  int rpre = ry + 2 >= ny ? (ry + 2) % ny : ry + 2;  // row r + 2
#pragma unroll
  for (int l = 0; l < 9; ++l) Pop<P>::load(A.src, l, A, ry, col, vec, fa[l]);
  if (K > 1) {
    const int r1 = ry + 1 == ny ? 0 : ry + 1;
#pragma unroll
    for (int l = 0; l < 9; ++l) Pop<P>::load(A.src, l, A, r1, col, vec, fb[l]);
  }

  auto iteration = [&](int k, T(&cur)[9][V]) {
    const int slot = k & 1;  // LDS slot of row r-2, refilled with row r below
    // h of row r (Sec. II: h = sum_l f_l)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T hs = cur[0][v];
#pragma unroll
      for (int l = 1; l < 9; ++l) hs += cur[l][v];
      h0[1 + v] = hs;
    }
    h0[0] = from_left(h0[V]);
    h0[V + 1] = from_right(h0[1]);
#pragma unroll
    for (int v = 0; v < V; ++v) kr[v] = kn[v];
    if constexpr (KF) {
      // kappa of row r, used by the pressure of row r in the next iteration
      const T *kp = (const T *)A.kfield + (size_t)ry * ldx;
      if constexpr (V == 2) {
        if (vec) {
          const float2 kv = *(const float2 *)(kp + col[0]);
          kn[0] = kv.x;
          kn[1] = kv.y;
        } else {
          kn[0] = kp[col[0]];
          kn[1] = kp[col[1]];
        }
      } else {
        kn[0] = kp[col[0]];
      }
    }
    // row r-2 leaves the LDS slot that row r takes over
    T f2[9][V];
    if (k >= 4) {
#pragma unroll
      for (int l = 0; l < 9; ++l)
#pragma unroll
        for (int v = 0; v < V; ++v) f2[l][v] = hist[slot][l][V * lane + v];
    }
#pragma unroll
    for (int l = 0; l < 9; ++l)
#pragma unroll
      for (int v = 0; v < V; ++v) hist[slot][l][V * lane + v] = cur[l][v];
    // prefetch row r + 2 into the registers just freed
    if (k + 2 < K) {
#pragma unroll
      for (int l = 0; l < 9; ++l) Pop<P>::load(A.src, l, A, rpre, col, vec, cur[l]);
    }

    if (k >= 2) {
      // film pressure of row r-1 (eqs. "pfilm", "disjoiningP", "n_laplace")
#pragma unroll
      for (int v = 0; v < V; ++v) {
        T odd = h1[v + 2];
        odd += h0[v + 1];
        odd += h1[v];
        odd += h2[v + 1];
        T even = h0[v + 2];
        even += h0[v];
        even += h2[v];
        even += h2[v + 2];
        const T hc = h1[v + 1];
        const T lap = (T(4) * odd + even - T(20) * hc) * T(1.0 / 6.0);
        const T rr = hstar / hc;
        const T phi = ipow(rr, n_exp) - ipow(rr, m_exp);
        const T kap = KF ? kr[v] : kap0;
        p1[v + 1] = -gamma * (lap + kap * phi);
      }
      p1[0] = from_left(p1[V]);
      p1[V + 1] = from_right(p1[1]);
    }

    if (k >= 4) {
      // collision and streaming of row y = r-2
      const int y = y0 + (k - 4);
      const int yN = (y + 1 == ny) ? 0 : y + 1;
      const int yS = (y == 0) ? ny - 1 : y - 1;
      T post[9][V];
      T hv[V], jxv[V], jyv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // isotropic gradient of p (eq. "derivative")
        T gx = cA * p2[v + 2];
        gx += cD * p1[v + 2];
        gx -= cD * p1[v];
        gx -= cA * p2[v];
        gx -= cD * p3[v];
        gx += cD * p3[v + 2];
        T gy = cD * p1[v + 2];
        gy += cA * p1[v + 1];
        gy += cD * p1[v];
        gy -= cD * p3[v];
        gy -= cA * p3[v + 1];
        gy -= cD * p3[v + 2];

        const T h = h2[1 + v];
        T jx = f2[1][v];
        jx += f2[2][v];
        jx -= f2[4][v];
        jx -= f2[5][v];
        jx -= f2[6][v];
        jx += f2[8][v];
        T jy = f2[2][v];
        jy += f2[3][v];
        jy += f2[4][v];
        jy -= f2[6][v];
        jy -= f2[7][v];
        jy -= f2[8][v];
        const T inv_h = T(1) / h;
        const T ux = jx * inv_h, uy = jy * inv_h;

        // forces (eqs. "force", "forcefric", "alphafric")
        const T alpha = (T(6) * h) / (T(2) * h * h + six_delta * h + three_delta2);
        const T fric = nu * alpha;
        const T Fx = -h * gx - fric * ux + h * ax;
        const T Fy = -h * gy - fric * uy + h * ay;

        // equilibrium (eq. "equilibria", lattice speed 1 in the denominators)
        const T usq = ux * ux + uy * uy;
        const T gh2 = g * h * h;
        const T hus = h * usq;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          T feq;
          const T cu = T(kCx[l]) * ux + T(kCy[l]) * uy;
          if (l == 0) {
            feq = h - gh2 * T(5.0 / 6.0) - hus * T(2.0 / 3.0);
          } else if (l & 1) {
            feq = gh2 * T(1.0 / 6.0) + h * cu * T(1.0 / 3.0) + h * cu * cu * T(0.5) - hus * T(1.0 / 6.0);
          } else {
            feq = gh2 * T(1.0 / 24.0) + h * cu * T(1.0 / 12.0) + h * cu * cu * T(0.125) - hus * T(1.0 / 24.0);
          }
          const T src = T(kW[l] / kCs2) * (T(kCx[l]) * Fx + T(kCy[l]) * Fy);
          post[l][v] = f2[l][v] + omega * (feq - f2[l][v]) + src;
        }
        hv[v] = h;
        jxv[v] = jx;
        jyv[v] = jy;
        if (out[v] && !(h > T(0) && h < T(INFINITY))) bad = 1;
      }

      // streaming: post-collision f_l(x) goes to x + c_l
      if constexpr (P == kF64) {
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          const int cx = kCx[l], cy = kCy[l];
          const int yd = cy == 0 ? y : (cy > 0 ? yN : yS);
          double *pl = (double *)(A.dst + plane_offset<P>(l, A.plane)) + (size_t)yd * ldx;
          const int xd = cx == 0 ? col[0] : (cx > 0 ? colE[0] : colW[0]);
          if (out[0]) pl[xd] = post[l][0];
        }
      } else {
        // FP32 values (FP32 form) or FP16 codes (FP16S form) of the moving
        // populations; the FP16S rest population absorbs their rounding
        float rest[V];
        if constexpr (P == kF16S) {
#pragma unroll
          for (int v = 0; v < V; ++v) rest[v] = hv[v];
        }
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          if (P == kF16S && l == 0) continue;
          const int cx = kCx[l], cy = kCy[l];
          const int yd = cy == 0 ? y : (cy > 0 ? yN : yS);
          using E = typename std::conditional<P == kF32, float, __half>::type;
          E e[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if constexpr (P == kF32) {
              e[v] = post[l][v];
            } else {
              const float s = (float)A.shift[l];
              e[v] = __float2half_rn((post[l][v] - s) * A.qscale);
              rest[v] -= s + __half2float(e[v]) * A.qinv;
            }
          }
          E *pl = (E *)(A.dst + plane_offset<P>(l, A.plane)) + (size_t)yd * ldx;
          if (pairs) {
            if (cx == 0) {
              store_pair<E>(pl, col[0], e[0], e[1], out[0], out[1]);
            } else if (cx > 0) {
              E left;
              if constexpr (P == kF32) left = from_left(e[1]);
              else left = half_from_left(e[1]);
              store_pair<E>(pl, col[0], left, e[0], srcE0, out[0]);
            } else {
              E right;
              if constexpr (P == kF32) right = from_right(e[0]);
              else right = half_from_right(e[0]);
              store_pair<E>(pl, col[0], e[1], right, out[1], srcW1);
            }
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
              const int xd = cx == 0 ? col[v] : (cx > 0 ? colE[v] : colW[v]);
              if (out[v]) pl[xd] = e[v];
            }
          }
        }
        if constexpr (P == kF16S) {
          float *pl = (float *)A.dst + (size_t)y * ldx;
          if (pairs) {
            store_pair<float>(pl, col[0], rest[0], rest[1], out[0], out[1]);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
              if (out[v]) pl[col[v]] = rest[v];
          }
        }
      }
      if constexpr (CAP) {
        T *cp = (T *)A.capture + (size_t)y * ldx;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (out[v]) {
            cp[col[v]] = hv[v];
            cp[A.plane + col[v]] = jxv[v];
            cp[2 * A.plane + col[v]] = jyv[v];
          }
        }
      }
    }

#pragma unroll
    for (int v = 0; v < V + 2; ++v) {
      h2[v] = h1[v];
      h1[v] = h0[v];
      p3[v] = p2[v];
      p2[v] = p1[v];
    }
    ry = ry + 1 == ny ? 0 : ry + 1;
    rpre = rpre + 1 == ny ? 0 : rpre + 1;
  };

  for (int k = 0; k < K; k += 2) {
    iteration(k, fa);
    if (k + 1 < K) iteration(k + 1, fb);
  }

  const unsigned long long m = __ballot(bad);
  if (m != 0ull && lane == __ffsll((unsigned long long)m) - 1) atomicOr(A.flag, 1);
}

// ---- initial populations and kappa ------------------------------------------
// f_l = f_l^eq(h0, u = 0): h0 - 5 g h0^2/6 (rest), g h0^2/6 (axes), g h0^2/24
// (diagonals); kappa = (1 - cos theta)(n - 1)(m - 1)/((n - m) h_*) (Sec. II).
template <int P>
__global__ void init_kernel(StepArgs A, const double *h0, const double *theta, double kconst) {
  using T = typename Form<P>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const double h = h0[(size_t)y * A.nx + x];
  const size_t o = (size_t)y * A.ldx + x;
  if (!(h > 0.0 && h < INFINITY)) atomicOr(A.flag, 1);
  const double gh2 = A.g * h * h;
  double e[9];
  e[0] = h - gh2 * (5.0 / 6.0);
  for (int l = 1; l < 9; ++l) e[l] = (l & 1) ? gh2 * (1.0 / 6.0) : gh2 * (1.0 / 24.0);
  char *d = A.dst;
  if constexpr (P == kF64 || P == kF32) {
    for (int l = 0; l < 9; ++l) ((T *)(d + plane_offset<P>(l, A.plane)))[o] = (T)e[l];
  } else {
    float sumdq = 0.f;
    for (int l = 1; l < 9; ++l) {
      const float s = (float)A.shift[l];
      const __half q = __float2half_rn(((float)e[l] - s) * A.qscale);
      ((__half *)(d + plane_offset<P>(l, A.plane)))[o] = q;
      sumdq += s + __half2float(q) * A.qinv;
    }
    ((float *)d)[o] = (float)h - sumdq;
  }
  if (theta != nullptr) {
    const double th = theta[(size_t)y * A.nx + x];
    ((T *)A.kfield)[o] = (T)((1.0 - cos(th)) * kconst);
  }
}

// ---- readout: h and u = j/h in FP64 from the stored populations --------------
template <int P>
__device__ __forceinline__ double pop_value(const char *buf, int l, const StepArgs &A, size_t o) {
  if constexpr (P == kF64) return ((const double *)(buf + plane_offset<P>(l, A.plane)))[o];
  else if constexpr (P == kF32) return (double)((const float *)(buf + plane_offset<P>(l, A.plane)))[o];
  else {
    if (l == 0) return (double)((const float *)buf)[o];
    const __half q = ((const __half *)(buf + plane_offset<P>(l, A.plane)))[o];
    return (double)((float)A.shift[l] + __half2float(q) * A.qinv);
  }
}

template <int P>
__global__ void read_kernel(StepArgs A, double *hout, double *uxo, double *uyo) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const size_t o = (size_t)y * A.ldx + x;
  double f[9];
  for (int l = 0; l < 9; ++l) f[l] = pop_value<P>(A.src, l, A, o);
  double h = f[0];
  for (int l = 1; l < 9; ++l) h += f[l];
  const double jx = f[1] + f[2] - f[4] - f[5] - f[6] + f[8];
  const double jy = f[2] + f[3] + f[4] - f[6] - f[7] - f[8];
  const size_t od = (size_t)y * A.nx + x;
  if (hout) hout[od] = h;
  if (uxo) uxo[od] = jx / h;
  if (uyo) uyo[od] = jy / h;
}

// ---- mass: deterministic two-pass FP64 reduction ------------------------------
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
    const int y = (int)(i / A.nx), x = (int)(i % A.nx);
    const size_t o = (size_t)y * A.ldx + x;
    double s = 0.0;
    for (int l = 0; l < 9; ++l) s += pop_value<P>(A.src, l, A, o);
    acc += s;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void mass_final_kernel(const double *partial, int np, double *out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---- launchers -----------------------------------------------------------------
template <int P>
static hipError_t launch_step_p(const StepArgs &A, bool kf, bool cap, hipStream_t s) {
  const dim3 grid(8 * A.per_xcd), block(64);
  if (kf) {
    if (cap) step_kernel<P, true, true><<<grid, block, 0, s>>>(A);
    else step_kernel<P, true, false><<<grid, block, 0, s>>>(A);
  } else {
    if (cap) step_kernel<P, false, true><<<grid, block, 0, s>>>(A);
    else step_kernel<P, false, false><<<grid, block, 0, s>>>(A);
  }
  return hipGetLastError();
}

hipError_t launch_step(int prec, const StepArgs &A, bool kf, bool cap, hipStream_t s) {
  switch (prec) {
    case kF64: return launch_step_p<kF64>(A, kf, cap, s);
    case kF32: return launch_step_p<kF32>(A, kf, cap, s);
    default: return launch_step_p<kF16S>(A, kf, cap, s);
  }
}

int step_columns_per_strip(int prec) {
  return prec == kF64 ? 64 * Form<kF64>::V - 4 : 64 * Form<kF32>::V - 4;
}

hipError_t launch_init(int prec, const StepArgs &A, const double *h0, const double *theta, double kconst,
                       hipStream_t s) {
  const dim3 block(256), grid((A.nx + 255) / 256, A.ny);
  switch (prec) {
    case kF64: init_kernel<kF64><<<grid, block, 0, s>>>(A, h0, theta, kconst); break;
    case kF32: init_kernel<kF32><<<grid, block, 0, s>>>(A, h0, theta, kconst); break;
    default: init_kernel<kF16S><<<grid, block, 0, s>>>(A, h0, theta, kconst); break;
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
  mass_final_kernel<<<1, 256, 0, s>>>(partial, np, out);
  return hipGetLastError();
}

}  // namespace tflbm
