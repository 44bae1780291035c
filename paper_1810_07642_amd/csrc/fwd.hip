// Forward kernels of the thin-film lattice Boltzmann method (arXiv:1810.07642,
// Sec. II): initial populations, the fused time step, readout of h and u, and
// the FP64 mass reduction.
//
// Layout (HBM): population records of B consecutive columns of a row, all
// nine populations of the record contiguous, two buffers ping-pong (see
// device.h).  Population l of site (x, y) is stored in row y at column
// x - c_lx: streaming in y is a push (a row writes into rows y - 1, y, y + 1)
// and streaming in x is a pull (each lane reads its left or right
// neighbour's value), so every lane stores exactly its own columns and every
// store of a wavefront covers whole 128-byte lines of a record.
//
// Fused step: one wavefront owns one record column (B output columns) plus a
// halo of (64 V - B)/2 columns per side, and a chunk of H rows, and marches
// down the rows.  Per row it reads the nine segments of the row's records
// (coalesced, prefetched two rows ahead), assembles the populations of its
// own columns (x shift through a cross-lane move), forms h; one row later the
// film pressure of the previous row (Laplacian of h and disjoining term); one
// more row later the isotropic pressure gradient, forces, equilibrium and
// collision of the row two above, whose populations were parked in LDS, and
// stores them.  Stencil neighbours in x come from adjacent lanes; the
// three-row windows of h and p stay in registers.  HBM sees each record read
// once and written once per step; the halo columns and the four halo rows of
// a chunk are re-read from L2.
#include <type_traits>

#include "device.h"
#include "launch.h"

namespace tflbm {

// Loads the stored values of population l at the lane's columns of one row
// (resource `row`); oe/o16 are the lane's byte offsets in a segment of the
// working type (FP32 or FP64) and in an FP16 segment; the segment offset is a
// compile-time immediate.
template <int P>
__device__ __forceinline__ void load_raw(rsrc_t row, int l, const int *oe, const int *o16, bool vec,
                                         typename Form<P>::T *out, const StepArgs &A) {
  constexpr int V = Form<P>::V;
  const int seg = seg_offset<P>(l);
  if constexpr (P == kF64) {
    out[0] = ld_f64(row, oe[0] + seg);
  } else if constexpr (P == kF32) {
    if (vec) {
      const float2 v = ld_f32x2(row, oe[0] + seg);
      out[0] = v.x;
      out[1] = v.y;
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) out[v] = ld_f32(row, oe[v] + seg);
    }
  } else {
    if (l == 0) {
      if (vec) {
        const float2 v = ld_f32x2(row, oe[0] + seg);
        out[0] = v.x;
        out[1] = v.y;
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = ld_f32(row, oe[v] + seg);
      }
    } else {
      const float s = (float)A.shift[l];
      if (vec) {
        const __half2 q = ld_f16x2(row, o16[0] + seg);
        out[0] = s + __low2float(q) * A.qinv;
        out[1] = s + __high2float(q) * A.qinv;
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = s + __half2float(ld_f16(row, o16[v] + seg)) * A.qinv;
      }
    }
  }
}

template <int P, bool KF, bool CAP>
__global__ __launch_bounds__(64) void step_kernel(StepArgs A) {
  using T = typename Form<P>::T;
  constexpr int V = Form<P>::V;
  constexpr int B = Form<P>::B;
  constexpr int RB = Form<P>::RB;
  constexpr int HX = (64 * V - B) / 2;  // halo columns per side
  constexpr int ES = sizeof(T);  // bytes per element of the FP32/FP64 segments and plane arrays
  // assembled populations of rows r-1 and r-2, each lane's own columns
  __shared__ T hist[2][9][64 * V];

  // XCD-aware tile order: consecutive workgroups land on different XCDs
  // (round robin), so give each XCD a contiguous block of tiles.
  const int b = blockIdx.x;
  const int tile = (b & 7) * A.per_xcd + (b >> 3);
  if (tile >= A.ntiles) return;
  const int strip = tile % A.nstrips;
  const int chunk = tile / A.nstrips;
  const int x0 = strip * B;
  const int y0 = chunk * A.H;
  const int yend = min(y0 + A.H, A.ny);
  const int xend = min(x0 + B, A.nx);
  const int lane = threadIdx.x;
  const int nx = A.nx, ny = A.ny, ldx = A.ldx;
  const size_t rowB = (size_t)A.nblk * RB;
  const uint32_t planeRowB = (uint32_t)(ldx * ES);  // one row of a plane array

  const int a = x0 - HX + V * lane;  // first (unwrapped) column of this lane
  // column, and its byte offset inside a row of records in a segment of the
  // working type (oe) and in an FP16 segment (o16)
  int col[V], oe[V], o16[V];
  bool out[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    col[v] = wrap(a + v, nx);
    const int blk = col[v] / B;
    const int pos = col[v] - blk * B;
    oe[v] = blk * RB + pos * ES;
    o16[v] = blk * RB + pos * 2;
    out[v] = (a + v >= x0) && (a + v < xend);
  }
  // vector access of the lane's column pair: both in one record, 8-byte aligned
  bool vec = true;
  bool vecp = true;  // same for the plane arrays (kappa, capture)
  if constexpr (V == 2) {
    vec = (col[1] == col[0] + 1) && (col[0] / B == col[1] / B) && ((col[0] & 1) == 0);
    vecp = (col[1] == col[0] + 1) && ((col[0] & 1) == 0);
  }

  const T omega = (T)A.omega, gamma = (T)A.gamma, nu = (T)A.nu, hstar = (T)A.hstar;
  const T ax = (T)A.ax, ay = (T)A.ay, g = (T)A.g;
  const T kap0 = (T)A.kappa0;
  const T cA = (T)(3.0 * kW[1]), cD = (T)(3.0 * kW[2]);  // gradient stencil weights
  const T three_delta2 = (T)(3.0 * A.delta * A.delta), six_delta = (T)(6.0 * A.delta);
  const T mgam = -gamma, mgam6 = (T)(-A.gamma / 6.0), om1 = (T)(1.0 - A.omega);
  const T g6 = (T)(A.g / 6.0), g24 = (T)(A.g / 24.0), g56 = (T)(5.0 * A.g / 6.0);
  const int n_exp = A.n_exp, m_exp = A.m_exp;

  T fa[9][V], fb[9][V];  // stored values of rows r (being consumed) and r + 1
  T h0[V + 2], h1[V + 2], h2[V + 2];
  T p1[V + 2], p2[V + 2], p3[V + 2];
  T kn[V], kr[V];
  int bad = 0;

  auto rsrc_src = [&](int row) { return make_rsrc(A.src + row * rowB, (uint32_t)rowB); };
  auto rsrc_dst = [&](int row) { return make_rsrc(A.dst + row * rowB, (uint32_t)rowB); };
  const int K = (yend - y0) + 4;
  int ry = wrap(y0 - 2, ny);                            // row r
  int rpre = ry + 2 >= ny ? (ry + 2) % ny : ry + 2;     // row r + 2
#pragma unroll
  for (int l = 0; l < 9; ++l) load_raw<P>(rsrc_src(ry), l, oe, o16, vec, fa[l], A);
  if (K > 1) {
    const int r1 = ry + 1 == ny ? 0 : ry + 1;
#pragma unroll
    for (int l = 0; l < 9; ++l) load_raw<P>(rsrc_src(r1), l, oe, o16, vec, fb[l], A);
  }

  auto iteration = [&](int k, T(&cur)[9][V]) {
    const int slot = k & 1;  // LDS slot of row r-2, refilled with row r below
    // populations of the lane's own columns: f_l(x) is stored at x - c_lx
    T f[9][V];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      if (kCx[l] == 0) {
#pragma unroll
        for (int v = 0; v < V; ++v) f[l][v] = cur[l][v];
      } else if (kCx[l] > 0) {
        f[l][0] = from_left(cur[l][V - 1]);
#pragma unroll
        for (int v = 1; v < V; ++v) f[l][v] = cur[l][v - 1];
      } else {
#pragma unroll
        for (int v = 0; v < V - 1; ++v) f[l][v] = cur[l][v + 1];
        f[l][V - 1] = from_right(cur[l][0]);
      }
    }
    // h of row r (Sec. II: h = sum_l f_l)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T hs = f[0][v];
#pragma unroll
      for (int l = 1; l < 9; ++l) hs += f[l][v];
      h0[1 + v] = hs;
    }
    h0[0] = from_left(h0[V]);
    h0[V + 1] = from_right(h0[1]);
#pragma unroll
    for (int v = 0; v < V; ++v) kr[v] = kn[v];
    if constexpr (KF) {
      // kappa of row r, used by the pressure of row r in the next iteration
      const rsrc_t kr_row = make_rsrc((const char *)A.kfield + (size_t)ry * planeRowB, planeRowB);
      if constexpr (V == 2) {
        if (vecp) {
          const float2 kv = ld_f32x2(kr_row, col[0] * 4);
          kn[0] = kv.x;
          kn[1] = kv.y;
        } else {
          kn[0] = ld_f32(kr_row, col[0] * 4);
          kn[1] = ld_f32(kr_row, col[1] * 4);
        }
      } else {
        kn[0] = ld_f64(kr_row, col[0] * 8);
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
      for (int v = 0; v < V; ++v) hist[slot][l][V * lane + v] = f[l][v];
    // prefetch row r + 2 into the registers just freed
    if (k + 2 < K) {
#pragma unroll
      for (int l = 0; l < 9; ++l) load_raw<P>(rsrc_src(rpre), l, oe, o16, vec, cur[l], A);
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
        // 6 lap = 4 sum_axes + sum_diagonals - 20 h
        const T lap6 = madd(T(-20), hc, madd(T(4), odd, even));
        const T phi = disjoining(hstar * recip(hc), n_exp, m_exp);
        const T kap = KF ? kr[v] : kap0;
        p1[v + 1] = madd(mgam6, lap6, mgam * kap * phi);
      }
      p1[0] = from_left(p1[V]);
      p1[V + 1] = from_right(p1[1]);
    }

    if (k >= 4) {
      // collision of row y = r-2, streamed into rows y-1, y, y+1
      const int y = y0 + (k - 4);
      const int yN = (y + 1 == ny) ? 0 : y + 1;
      const int yS = (y == 0) ? ny - 1 : y - 1;
      T post[9][V];
      T hv[V], jxv[V], jyv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // isotropic gradient of p (eq. "derivative"): axis weight 1/3, diagonal 1/12
        const T gx = madd(cA, p2[v + 2] - p2[v], cD * ((p1[v + 2] - p1[v]) + (p3[v + 2] - p3[v])));
        const T gy = madd(cA, p1[v + 1] - p3[v + 1], cD * ((p1[v + 2] - p3[v + 2]) + (p1[v] - p3[v])));

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
        const T inv_h = recip(h);
        const T ux = jx * inv_h, uy = jy * inv_h;

        // forces (eqs. "force", "forcefric", "alphafric"):
        // F = h (a - grad p) - nu alpha(h) u, alpha = 6 h / (2 h^2 + 6 delta h + 3 delta^2)
        const T alpha = T(6) * h * recip(madd(T(2) * h, h, madd(six_delta, h, three_delta2)));
        const T fric = nu * alpha;
        const T Fx = madd(h, ax - gx, -fric * ux);
        const T Fy = madd(h, ay - gy, -fric * uy);

        // equilibrium (eq. "equilibria", lattice speed 1 in the denominators),
        // written as h times a polynomial in c.u:
        //   rest: h (1 - 5 g h/6 - 2 u^2/3)
        //   axes: h ((g h - u^2)/6 + c.u/3 + (c.u)^2/2)
        //   diagonals: h ((g h - u^2)/24 + c.u/12 + (c.u)^2/8)
        // and BGK with forcing, post = f + omega (feq - f) + 3 w_l c_l.F
        const T usq = madd(ux, ux, uy * uy);
        const T a1 = madd(g6, h, usq * T(-1.0 / 6.0));
        const T a2 = madd(g24, h, usq * T(-1.0 / 24.0));
        const T hom = h * omega;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          T poly, src;
          if (l == 0) {
            poly = madd(-g56, h, madd(usq, T(-2.0 / 3.0), T(1)));
            src = T(0);
          } else {
            const int cx = kCx[l], cy = kCy[l];
            const T cu = cx == 0 ? (cy > 0 ? uy : -uy)
                                 : (cy == 0 ? (cx > 0 ? ux : -ux)
                                            : (cx > 0 ? (cy > 0 ? ux + uy : ux - uy) : (cy > 0 ? uy - ux : -ux - uy)));
            const T cF = cx == 0 ? (cy > 0 ? Fy : -Fy)
                                 : (cy == 0 ? (cx > 0 ? Fx : -Fx)
                                            : (cx > 0 ? (cy > 0 ? Fx + Fy : Fx - Fy) : (cy > 0 ? Fy - Fx : -Fx - Fy)));
            if (l & 1) {
              poly = madd(cu, madd(cu, T(0.5), T(1.0 / 3.0)), a1);
              src = cF * T(1.0 / 3.0);
            } else {
              poly = madd(cu, madd(cu, T(0.125), T(1.0 / 12.0)), a2);
              src = cF * T(1.0 / 12.0);
            }
          }
          // f + omega (h poly - f) + src = (1 - omega) f + (h omega) poly + src
          post[l][v] = madd(om1, f2[l][v], madd(hom, poly, src));
        }
        hv[v] = h;
        jxv[v] = jx;
        jyv[v] = jy;
        if (out[v] && !(h > T(0) && h < T(INFINITY))) bad = 1;
      }

      // streaming: the post-collision f_l of site (x, y) goes to stored
      // column x of row y + c_ly
      const bool pair = out[0] && out[V - 1] && vec;
      const rsrc_t rowD[3] = {rsrc_dst(yS), rsrc_dst(y), rsrc_dst(yN)};  // indexed by c_ly + 1
      if constexpr (P == kF16S) {
        float rest[V];
#pragma unroll
        for (int v = 0; v < V; ++v) rest[v] = hv[v];
#pragma unroll
        for (int l = 1; l < 9; ++l) {
          const rsrc_t rd = rowD[kCy[l] + 1];
          const int seg = seg_offset<P>(l);
          const float s = (float)A.shift[l];
          __half q[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            q[v] = __float2half_rn((post[l][v] - s) * A.qscale);
            rest[v] -= s + __half2float(q[v]) * A.qinv;  // rest population absorbs the rounding
          }
          if (pair) {
            st_f16x2(rd, o16[0] + seg, q[0], q[1]);
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
              if (out[v]) st_f16(rd, o16[v] + seg, q[v]);
          }
        }
        if (pair) {
          st_f32x2(rowD[1], oe[0], rest[0], rest[1]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (out[v]) st_f32(rowD[1], oe[v], rest[v]);
        }
        // fill the 64-byte pads after the c_ly = +1 and -1 groups of a full
        // record so that its lines are written whole
        if (xend - x0 == B) {
          const int q16 = lane - HX / V;
          if (q16 >= 0 && q16 < 16) {
            const int rec = (x0 / B) * RB;
            st_f32(rowD[2], rec + 1344 + 4 * q16, 0.f);
            st_f32(rowD[0], rec + 1984 + 4 * q16, 0.f);
          }
        }
      } else {
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          const rsrc_t rd = rowD[kCy[l] + 1];
          const int seg = seg_offset<P>(l);
          if constexpr (P == kF64) {
            if (out[0]) st_f64(rd, oe[0] + seg, post[l][0]);
          } else {
            if (pair) {
              st_f32x2(rd, oe[0] + seg, post[l][0], post[l][1]);
            } else {
#pragma unroll
              for (int v = 0; v < V; ++v)
                if (out[v]) st_f32(rd, oe[v] + seg, post[l][v]);
            }
          }
        }
      }
      if constexpr (CAP) {
        const size_t ro = (size_t)y * planeRowB;
        const rsrc_t c0 = make_rsrc(A.capture + ro, planeRowB);
        const rsrc_t c1 = make_rsrc(A.capture + (size_t)A.plane * ES + ro, planeRowB);
        const rsrc_t c2 = make_rsrc(A.capture + 2 * (size_t)A.plane * ES + ro, planeRowB);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (out[v]) {
            st_t(c0, col[v] * ES, hv[v]);
            st_t(c1, col[v] * ES, jxv[v]);
            st_t(c2, col[v] * ES, jyv[v]);
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
template <int P> __device__ __forceinline__ char *pop_ptr(char *buf, int l, int y, int c, const StepArgs &A) {
  constexpr int B = Form<P>::B;
  const int blk = c / B, pos = c - blk * B;
  char *rec = buf + ((size_t)y * A.nblk + blk) * Form<P>::RB + seg_offset<P>(l);
  const int es = (P == kF64) ? 8 : ((P == kF16S && l != 0) ? 2 : 4);
  return rec + (size_t)pos * es;
}

template <int P>
__global__ void init_kernel(StepArgs A, const double *h0, const double *theta, double kconst) {
  using T = typename Form<P>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const double h = h0[(size_t)y * A.nx + x];
  if (!(h > 0.0 && h < INFINITY)) atomicOr(A.flag, 1);
  const double gh2 = A.g * h * h;
  double e[9];
  e[0] = h - gh2 * (5.0 / 6.0);
  for (int l = 1; l < 9; ++l) e[l] = (l & 1) ? gh2 * (1.0 / 6.0) : gh2 * (1.0 / 24.0);
  if constexpr (P == kF64 || P == kF32) {
    for (int l = 0; l < 9; ++l) *(T *)pop_ptr<P>(A.dst, l, y, wrap(x - kCx[l], A.nx), A) = (T)e[l];
  } else {
    float sumdq = 0.f;
    for (int l = 1; l < 9; ++l) {
      const float s = (float)A.shift[l];
      const __half q = __float2half_rn(((float)e[l] - s) * A.qscale);
      *(__half *)pop_ptr<P>(A.dst, l, y, wrap(x - kCx[l], A.nx), A) = q;
      sumdq += s + __half2float(q) * A.qinv;
    }
    *(float *)pop_ptr<P>(A.dst, 0, y, x, A) = (float)h - sumdq;
  }
  if (theta != nullptr) {
    const double th = theta[(size_t)y * A.nx + x];
    ((T *)A.kfield)[(size_t)y * A.ldx + x] = (T)((1.0 - cos(th)) * kconst);
  }
}

// ---- readout: h and u = j/h in FP64 from the stored populations --------------
template <int P>
__global__ void read_kernel(StepArgs A, double *hout, double *uxo, double *uyo) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  double f[9];
  for (int l = 0; l < 9; ++l) f[l] = (double)pop_at<P>(A.src, l, y, wrap(x - kCx[l], A.nx), A);
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
    const int y = (int)(i / A.nx), c = (int)(i % A.nx);
    double s = 0.0;
    for (int l = 0; l < 9; ++l) s += (double)pop_at<P>(A.src, l, y, c, A);
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

int record_sites(int prec) { return prec == kF64 ? Form<kF64>::B : Form<kF32>::B; }
int record_bytes(int prec) {
  return prec == kF64 ? Form<kF64>::RB : (prec == kF32 ? Form<kF32>::RB : Form<kF16S>::RB);
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
