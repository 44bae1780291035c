// Reverse mode of the thin-film lattice Boltzmann step: the hand-written
// vector-Jacobian product of one step of eq. "LBE" (arXiv:1810.07642, Sec. II)
// with respect to the pre-collision populations and the kappa field.
//
// Notation.  Forward step t, at every site x (pre-collision state f):
//   h = sum_l f_l, j = sum_l c_l f_l, u = j/h
//   p = -gamma (L h + kappa phi(h)),  phi(h) = (h_*/h)^n - (h_*/h)^m
//   G = grad_s p (isotropic gradient),  F = -h G - nu alpha(h) u + h a
//   f*_l = f_l + omega (feq_l(h, u) - f_l) + 3 w_l c_l . F,   f_l(x + c_l, t + 1) = f*_l(x).
// Adjoint.  lambda^t_l(x) = dLoss/df^t_l(x).  The stored adjoint is
// pre-shifted, mu_l(x) = lambda^{t+1}_l(x + c_l) = dLoss/df*_l(x), so that
// all nine values a site needs are at the site itself (the same footprint as
// the forward push layout).  One reverse step computes, at every site:
//   Lambda_F = 3 sum_l w_l c_l mu_l                       (from the source term)
//   lambda_G = -h Lambda_F                                (from F = -h G)
//   lambda_p = -div_s lambda_G                            (grad_s^T = -div_s)
//   lambda_u = omega sum_l mu_l dfeq_l/du - nu alpha Lambda_F
//   lambda_h = omega sum_l mu_l dfeq_l/dh + Lambda_F.(-G - nu alpha'(h) u + a)
//              - gamma L(lambda_p) - gamma kappa phi'(h) lambda_p - lambda_u.u/h    (L^T = L)
//   lambda_j = lambda_u / h
//   lambda^t_l = (1 - omega) mu_l + lambda_h + c_l . lambda_j
//   g_kappa += -gamma phi(h) lambda_p          (FP64 accumulation)
// and stores lambda^t_l(x) at x - c_l (the pre-shifted form for step t-1).
// The forward moments h, j of step t come from the capture written by the
// forward step; the film pressure and its gradient are recomputed from h.
#include <cstring>

#include "device.h"
#include "launch.h"
#include "sim.h"

namespace tflbm {

struct AdjArgs {
  const char *src;     // mu at the end of step t: [9][ny][ldx] in T
  char *dst;           // mu at the end of step t-1
  const char *cap;     // h, jx, jy of step t: capture records of the forward form
  const void *kfield;  // kappa [ny][ldx] in T or nullptr
  double *gk;          // dLoss/dkappa [ny][ldx] FP64
  int nx, ny, ldx;
  int cnblk;           // capture records per row (those of the forward step)
  int64_t plane;
  int nstrips, H, ntiles, per_xcd;
  int n_exp, m_exp;
  double omega, gamma, nu, hstar, delta, ax, ay, g, kappa0;
};

constexpr int kAdjOutW = 60;  // 64 lanes, one column each, two halo columns per side

// The forward form whose capture records the reverse step reads (FP32 and
// FP16S share the record geometry).
template <typename T> struct CapForm;
template <> struct CapForm<double> {
  static constexpr int B = Form<kF64>::B, CRB = cap_record_bytes<kF64>();
};
template <> struct CapForm<float> {
  static constexpr int B = Form<kF32>::B, CRB = cap_record_bytes<kF32>();
  static_assert(Form<kF16S>::B == Form<kF32>::B && cap_record_bytes<kF16S>() == cap_record_bytes<kF32>(),
                "FP32 and FP16S capture records must agree");
};
int adj_columns_per_strip() { return kAdjOutW; }

// Lambda_F = 3 sum_l w_l c_l mu_l through differences of opposite populations.
template <typename T>
__device__ __forceinline__ void lambda_force(const T (&mu)[9], T cA, T cD, T &LFx, T &LFy) {
  const T d15 = mu[1] - mu[5], d37 = mu[3] - mu[7], d26 = mu[2] - mu[6], d48 = mu[4] - mu[8];
  LFx = madd(cA, d15, cD * (d26 - d48));
  LFy = madd(cA, d37, cD * (d26 + d48));
}

// r^n and r^m; (9, 3) and (3, 9) without loops.
template <typename T> __device__ __forceinline__ void powers(T r, int n, int m, T &rn, T &rm) {
  if ((n == 9 && m == 3) || (n == 3 && m == 9)) {
    const T r3 = r * r * r;
    const T r9 = r3 * r3 * r3;
    rn = n == 9 ? r9 : r3;
    rm = n == 9 ? r3 : r9;
  } else {
    rn = ipow(r, n);
    rm = ipow(r, m);
  }
}

template <typename T, bool KF>
__global__ __launch_bounds__(64) void adj_step_kernel(AdjArgs A) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * A.per_xcd + (b >> 3);
  if (tile >= A.ntiles) return;
  const int strip = tile % A.nstrips;
  const int chunk = tile / A.nstrips;
  const int x0 = strip * kAdjOutW;
  const int y0 = chunk * A.H;
  const int yend = min(y0 + A.H, A.ny);
  const int xend = min(x0 + kAdjOutW, A.nx);
  const int lane = threadIdx.x;
  const int nx = A.nx, ny = A.ny, ldx = A.ldx;
  const int64_t plane = A.plane;

  const int a = x0 - 2 + lane;
  const int col = wrap(a, nx), colE = wrap(a + 1, nx), colW = wrap(a - 1, nx);
  const bool out = (a >= x0) && (a < xend);

  const T omega = (T)A.omega, gamma = (T)A.gamma, nu = (T)A.nu, hstar = (T)A.hstar;
  const T delta = (T)A.delta, ax = (T)A.ax, ay = (T)A.ay, g = (T)A.g, kap0 = (T)A.kappa0;
  const T cA = (T)(3.0 * kW[1]), cD = (T)(3.0 * kW[2]);
  const int n_exp = A.n_exp, m_exp = A.m_exp;
  const T *mu_src = (const T *)A.src;
  // byte offset of this lane's column in a row of capture records
  constexpr int CB = CapForm<T>::B, CRB = CapForm<T>::CRB, CSEG = CB * (int)sizeof(T);
  const int crec = (col / CB) * CRB + (col % CB) * (int)sizeof(T);
  const size_t crow = (size_t)A.cnblk * CRB;

  // rolling rows: index 0 = row r (newest), 1 = r-1, 2 = r-2
  T mu0[9], mu1[9], mu2[9], mun[9];
  T hC0, hC1, hC2, hL0, hL1, hL2, hR0, hR1, hR2;        // h with left/right neighbours
  T jx0 = 0, jx1 = 0, jx2 = 0, jy0 = 0, jy1 = 0, jy2 = 0;
  T hn, jxn, jyn, kn = 0, k0 = 0, k1 = 0, k2 = 0;
  T LFx0 = 0, LFy0 = 0, LFx1 = 0, LFy1 = 0, LFx2 = 0, LFy2 = 0;  // Lambda_F of rows r, r-1, r-2
  T gxC0, gxL0, gxR0, gyC0, gyL0, gyR0;                  // lambda_G of rows r, r-1, r-2
  T gxC1, gxL1, gxR1, gyC1, gyL1, gyR1;
  T gxC2, gxL2, gxR2, gyC2, gyL2, gyR2;
  T pC1 = 0, pL1 = 0, pR1 = 0, pC2 = 0, pL2 = 0, pR2 = 0, pC3 = 0, pL3 = 0, pR3 = 0;   // p rows r-1, r-2, r-3
  T qC1 = 0, qL1 = 0, qR1 = 0, qC2 = 0, qL2 = 0, qR2 = 0, qC3 = 0, qL3 = 0, qR3 = 0;   // lambda_p rows r-1, r-2, r-3
  hC1 = hL1 = hR1 = hC2 = hL2 = hR2 = 0;
  gxC1 = gxL1 = gxR1 = gyC1 = gyL1 = gyR1 = 0;
  gxC2 = gxL2 = gxR2 = gyC2 = gyL2 = gyR2 = 0;
#pragma unroll
  for (int l = 0; l < 9; ++l) mu1[l] = mu2[l] = 0;

  const int K = (yend - y0) + 4;
  int ry = wrap(y0 - 2, ny);
  auto load_row = [&](int row) {
    const size_t o = (size_t)row * ldx + col;
#pragma unroll
    for (int l = 0; l < 9; ++l) mun[l] = mu_src[(size_t)l * plane + o];
    const char *cr = A.cap + (size_t)row * crow + crec;
    hn = *(const T *)cr;
    jxn = *(const T *)(cr + CSEG);
    jyn = *(const T *)(cr + 2 * CSEG);
    if constexpr (KF) kn = ((const T *)A.kfield)[o];
  };
  load_row(ry);

  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      mu2[l] = mu1[l];
      mu1[l] = mu0[l];
      mu0[l] = mun[l];
    }
    jx2 = jx1; jx1 = jx0; jx0 = jxn;
    jy2 = jy1; jy1 = jy0; jy0 = jyn;
    k2 = k1; k1 = k0; k0 = KF ? kn : kap0;
    hC2 = hC1; hL2 = hL1; hR2 = hR1;
    hC1 = hC0; hL1 = hL0; hR1 = hR0;
    hC0 = hn;
    LFx2 = LFx1; LFy2 = LFy1;
    LFx1 = LFx0; LFy1 = LFy0;
    gxC2 = gxC1; gxL2 = gxL1; gxR2 = gxR1; gyC2 = gyC1; gyL2 = gyL1; gyR2 = gyR1;
    gxC1 = gxC0; gxL1 = gxL0; gxR1 = gxR0; gyC1 = gyC0; gyL1 = gyL0; gyR1 = gyR0;
    const int rn = (ry + 1 == ny) ? 0 : ry + 1;
    if (k + 1 < K) load_row(rn);

    hL0 = from_left(hC0);
    hR0 = from_right(hC0);
    {
      // Lambda_F and lambda_G of row r
      lambda_force(mu0, cA, cD, LFx0, LFy0);
      gxC0 = -hC0 * LFx0;
      gyC0 = -hC0 * LFy0;
      gxL0 = from_left(gxC0);
      gxR0 = from_right(gxC0);
      gyL0 = from_left(gyC0);
      gyR0 = from_right(gyC0);
    }

    if (k >= 2) {
      // rotate p and lambda_p (rows r-1 computed now)
      pC3 = pC2; pL3 = pL2; pR3 = pR2;
      pC2 = pC1; pL2 = pL1; pR2 = pR1;
      qC3 = qC2; qL3 = qL2; qR3 = qR2;
      qC2 = qC1; qL2 = qL1; qR2 = qR1;
      // forward film pressure of row r-1 from h rows r-2 .. r
      const T odd = ((hR1 + hC0) + hL1) + hC2;
      const T even = ((hR0 + hL0) + hL2) + hR2;
      const T lap = (T(4) * odd + even - T(20) * hC1) * T(1.0 / 6.0);
      T rn1, rm1;
      powers(hstar * recip(hC1), n_exp, m_exp, rn1, rm1);
      pC1 = -gamma * (lap + k1 * (rn1 - rm1));
      pL1 = from_left(pC1);
      pR1 = from_right(pC1);
      // lambda_p of row r-1 = -div_s lambda_G (lambda_G rows r-2 .. r)
      T dx = cA * gxR1;
      dx += cD * gxR0;
      dx -= cD * gxL0;
      dx -= cA * gxL1;
      dx -= cD * gxL2;
      dx += cD * gxR2;
      T dy = cD * gyR0;
      dy += cA * gyC0;
      dy += cD * gyL0;
      dy -= cD * gyL2;
      dy -= cA * gyC2;
      dy -= cD * gyR2;
      qC1 = -(dx + dy);
      qL1 = from_left(qC1);
      qR1 = from_right(qC1);
    }

    if (k >= 4 && out) {
      // output row y = r-2: site quantities from row index 2
      const int y = y0 + (k - 4);
      const T h = hC2;
      const T inv_h = recip(h);
      const T ux = jx2 * inv_h, uy = jy2 * inv_h;
      // forward pressure gradient at y (p rows r-3 .. r-1)
      const T Gx = madd(cA, pR2 - pL2, cD * ((pR1 - pL1) + (pR3 - pL3)));
      const T Gy = madd(cA, pC1 - pC3, cD * ((pR1 - pR3) + (pL1 - pL3)));
      // Laplacian of lambda_p at y (lambda_p rows r-3 .. r-1)
      const T qodd = ((qR2 + qC1) + qL2) + qC3;
      const T qeven = ((qR1 + qL1) + qL3) + qR3;
      const T lapq = (T(4) * qodd + qeven - T(20) * qC2) * T(1.0 / 6.0);
      const T lp = qC2;

      const T three_d2 = T(3) * delta * delta;
      const T invD = recip(madd(T(2) * h, h, madd(T(6) * delta, h, three_d2)));
      const T alpha = T(6) * h * invD;
      const T dalpha = T(6) * madd(T(-2) * h, h, three_d2) * (invD * invD);
      T rn_, rm_;
      powers(hstar * inv_h, n_exp, m_exp, rn_, rm_);
      const T phi = rn_ - rm_;
      const T dphi = (T(m_exp) * rm_ - T(n_exp) * rn_) * inv_h;
      const T LFx = LFx2, LFy = LFy2;

      // omega sum_l mu_l dfeq_l/dh and omega sum_l mu_l dfeq_l/du over pairs
      // of opposite populations: S = mu_l + mu_-l takes the parts of the
      // derivatives even in c, D = mu_l - mu_-l the odd ones
      const T usq = madd(ux, ux, uy * uy);
      const T gh = g * h;
      const T up = ux + uy, um = uy - ux;
      const T S15 = mu2[1] + mu2[5], D15 = mu2[1] - mu2[5];
      const T S37 = mu2[3] + mu2[7], D37 = mu2[3] - mu2[7];
      const T S26 = mu2[2] + mu2[6], D26 = mu2[2] - mu2[6];
      const T S48 = mu2[4] + mu2[8], D48 = mu2[4] - mu2[8];
      // d/dh: rest 1 - 5gh/3 - 2u^2/3; axes gh/3 + cu/3 + cu^2/2 - u^2/6;
      // diagonals gh/12 + cu/12 + cu^2/8 - u^2/24
      T sh = mu2[0] * madd(gh, T(-5.0 / 3.0), madd(usq, T(-2.0 / 3.0), T(1)));
      sh = madd(S15 + S37, madd(gh, T(1.0 / 3.0), usq * T(-1.0 / 6.0)), sh);
      sh = madd(T(0.5), madd(S15, ux * ux, S37 * (uy * uy)), sh);
      sh = madd(T(1.0 / 3.0), madd(D15, ux, D37 * uy), sh);
      sh = madd(S26 + S48, madd(gh, T(1.0 / 12.0), usq * T(-1.0 / 24.0)), sh);
      sh = madd(T(0.125), madd(S26, up * up, S48 * (um * um)), sh);
      sh = madd(T(1.0 / 12.0), madd(D26, up, D48 * um), sh);
      // d/du = h (c1 c + c2 (c.u) c - c3 u): rest -4u/3; axes (1/3, 1, 1/3);
      // diagonals (1/12, 1/4, 1/12)
      T sx = mu2[0] * ux * T(-4.0 / 3.0);
      sx = madd(D15, T(1.0 / 3.0), sx);
      sx = madd(S15 - T(0.5) * S37, ux * T(2.0 / 3.0), sx);
      sx = madd(D26 - D48, T(1.0 / 12.0), sx);
      sx = madd(S26, madd(up, T(0.25), ux * T(-1.0 / 12.0)), sx);
      sx = madd(S48, madd(um, T(-0.25), ux * T(-1.0 / 12.0)), sx);
      T sy = mu2[0] * uy * T(-4.0 / 3.0);
      sy = madd(D37, T(1.0 / 3.0), sy);
      sy = madd(S37 - T(0.5) * S15, uy * T(2.0 / 3.0), sy);
      sy = madd(D26 + D48, T(1.0 / 12.0), sy);
      sy = madd(S26, madd(up, T(0.25), uy * T(-1.0 / 12.0)), sy);
      sy = madd(S48, madd(um, T(0.25), uy * T(-1.0 / 12.0)), sy);
      const T fric = nu * alpha;
      const T lux = madd(omega * h, sx, -fric * LFx);
      const T luy = madd(omega * h, sy, -fric * LFy);
      T lh = omega * sh + LFx * (-Gx - nu * dalpha * ux + ax) + LFy * (-Gy - nu * dalpha * uy + ay) -
             gamma * lapq - gamma * k2 * dphi * lp;
      lh -= (lux * ux + luy * uy) * inv_h;
      const T ljx = lux * inv_h, ljy = luy * inv_h;

      const int yN = (y + 1 == ny) ? 0 : y + 1;
      const int yS = (y == 0) ? ny - 1 : y - 1;
      T *dst = (T *)A.dst;
      const T om1 = T(1) - omega;
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        const int cx = kCx[l], cy = kCy[l];
        const T cl = cx == 0 ? (cy == 0 ? T(0) : (cy > 0 ? ljy : -ljy))
                             : (cy == 0 ? (cx > 0 ? ljx : -ljx)
                                        : (cx > 0 ? (cy > 0 ? ljx + ljy : ljx - ljy) : (cy > 0 ? ljy - ljx : -ljx - ljy)));
        const T lam = madd(om1, mu2[l], lh + cl);
        // store at x - c_l
        const int yd = cy == 0 ? y : (cy > 0 ? yS : yN);
        const int xd = cx == 0 ? col : (cx > 0 ? colW : colE);
        dst[(size_t)l * plane + (size_t)yd * ldx + xd] = lam;
      }
      double *gk = A.gk + (size_t)y * ldx + col;
      *gk += -(double)gamma * (double)phi * (double)lp;
    }
    ry = rn;
  }
}

// mu_l(x) = dLoss/dh_N(x + c_l) for every l; g_kappa = 0.
template <typename T>
__global__ void adj_seed_kernel(AdjArgs A, const double *grad_h) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  T *dst = (T *)A.dst;
  for (int l = 0; l < 9; ++l) {
    const int xs = wrap(x + kCx[l], A.nx), ys = wrap(y + kCy[l], A.ny);
    dst[(size_t)l * A.plane + (size_t)y * A.ldx + x] = (T)grad_h[(size_t)ys * A.nx + xs];
  }
  A.gk[(size_t)y * A.ldx + x] = 0.0;
}

// dLoss/dh0 = sum_l lambda^0_l dE_l/dh0 with lambda^0_l(x) = mu_l(x - c_l);
// dLoss/dtheta = dLoss/dkappa * (n-1)(m-1)/((n-m) h_*) * sin(theta).
template <typename T>
__global__ void adj_finish_kernel(AdjArgs A, const double *h0, const double *theta, double theta0, double kconst,
                                  double *grad_h0, double *grad_theta) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const size_t od = (size_t)y * A.nx + x;
  const T *src = (const T *)A.src;
  if (grad_h0) {
    const double h = h0[od];
    double s = 0.0;
    for (int l = 0; l < 9; ++l) {
      const int xs = wrap(x - kCx[l], A.nx), ys = wrap(y - kCy[l], A.ny);
      const double lam = (double)src[(size_t)l * A.plane + (size_t)ys * A.ldx + xs];
      const double dE = l == 0 ? 1.0 - A.g * h * (5.0 / 3.0) : ((l & 1) ? A.g * h / 3.0 : A.g * h / 12.0);
      s += lam * dE;
    }
    grad_h0[od] = s;
  }
  if (grad_theta) {
    const double th = theta ? theta[od] : theta0;
    grad_theta[od] = A.gk[(size_t)y * A.ldx + x] * kconst * sin(th);
  }
}

template <typename T>
static hipError_t adj_step_t(const AdjArgs &B, bool kf, hipStream_t s) {
  const dim3 grid(8 * B.per_xcd), block(64);
  if (kf) adj_step_kernel<T, true><<<grid, block, 0, s>>>(B);
  else adj_step_kernel<T, false><<<grid, block, 0, s>>>(B);
  return hipGetLastError();
}

hipError_t launch_adj_step(int prec, const AdjArgs &B, bool kf, hipStream_t s) {
  return prec == kF64 ? adj_step_t<double>(B, kf, s) : adj_step_t<float>(B, kf, s);
}

hipError_t launch_adj_seed(int prec, const AdjArgs &B, const double *grad_h, hipStream_t s) {
  const dim3 block(256), grid((B.nx + 255) / 256, B.ny);
  if (prec == kF64) adj_seed_kernel<double><<<grid, block, 0, s>>>(B, grad_h);
  else adj_seed_kernel<float><<<grid, block, 0, s>>>(B, grad_h);
  return hipGetLastError();
}

hipError_t launch_adj_finish(int prec, const AdjArgs &B, const double *h0, const double *theta, double theta0,
                             double kconst, double *grad_h0, double *grad_theta, hipStream_t s) {
  const dim3 block(256), grid((B.nx + 255) / 256, B.ny);
  if (prec == kF64)
    adj_finish_kernel<double><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
  else
    adj_finish_kernel<float><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
  return hipGetLastError();
}

static size_t adj_buf_bytes(const tflbm_sim *s) { return 9 * (size_t)s->plane * work_bytes(s->p.prec); }
static size_t round4k(size_t v) { return (v + 4095) / 4096 * 4096; }

static AdjArgs make_adj_args(const tflbm_sim *s, void *d_adj) {
  AdjArgs B;
  std::memset(&B, 0, sizeof(B));
  char *base = (char *)d_adj;
  const size_t nb = round4k(adj_buf_bytes(s));
  B.src = base + (s->adj_cur == 0 ? 0 : nb);
  B.dst = base + (s->adj_cur == 0 ? nb : 0);
  B.gk = (double *)(base + 2 * nb);
  B.kfield = s->kfield ? (const void *)(s->ws + s->off_k) : nullptr;
  B.nx = s->p.nx;
  B.ny = s->p.ny;
  B.ldx = s->ldx;
  B.cnblk = s->nblk;
  B.plane = s->plane;
  B.nstrips = s->adj_nstrips;
  B.H = s->adj_rows;
  B.ntiles = s->adj_ntiles;
  B.per_xcd = s->adj_per_xcd;
  B.n_exp = s->p.n_exp;
  B.m_exp = s->p.m_exp;
  B.omega = 1.0 / s->p.tau;
  B.gamma = s->p.gamma;
  B.nu = (s->p.tau - 0.5) / 3.0;
  B.hstar = s->p.hstar;
  B.delta = s->p.delta;
  B.ax = s->p.ax;
  B.ay = s->p.ay;
  B.g = s->p.g;
  B.kappa0 = s->kappa0;
  return B;
}

}  // namespace tflbm

using namespace tflbm;

extern "C" {

size_t tflbm_adj_bytes(const tflbm_sim *sim) {
  if (!sim) return 0;
  return 2 * round4k(adj_buf_bytes(sim)) + round4k(8 * (size_t)sim->plane);
}

int tflbm_adj_seed(tflbm_sim *sim, void *d_adj, const double *d_grad_h, tflbm_stream_t stream) {
  if (!sim || !d_adj || !d_grad_h || ((uintptr_t)d_adj & 255) != 0) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  sim->adj_cur = 1;  // seed writes the "dst" of a cur=1 state, i.e. the first buffer
  AdjArgs B = make_adj_args(sim, d_adj);
  const int rc = hip_status(sim, launch_adj_seed(sim->p.prec, B, d_grad_h, (hipStream_t)stream));
  if (rc) return rc;
  sim->adj_cur = 0;
  sim->adj_seeded = true;
  return TFLBM_OK;
}

int tflbm_adj_step(tflbm_sim *sim, void *d_adj, const void *d_capture_t, tflbm_stream_t stream) {
  if (!sim || !d_adj || !d_capture_t) return TFLBM_EINVAL;
  if (!sim->adj_seeded) return TFLBM_ESTATE;
  AdjArgs B = make_adj_args(sim, d_adj);
  B.cap = (const char *)d_capture_t;
  const int rc = hip_status(sim, launch_adj_step(sim->p.prec, B, sim->kfield, (hipStream_t)stream));
  if (rc) return rc;
  sim->adj_cur ^= 1;
  return TFLBM_OK;
}

int tflbm_adj_finish(tflbm_sim *sim, const void *d_adj, const double *d_h0, const double *d_theta,
                     double *d_grad_h0, double *d_grad_theta, tflbm_stream_t stream) {
  if (!sim || !d_adj) return TFLBM_EINVAL;
  if (d_grad_h0 && !d_h0) return TFLBM_EINVAL;
  if (!sim->adj_seeded) return TFLBM_ESTATE;
  AdjArgs B = make_adj_args(sim, (void *)d_adj);
  return hip_status(sim, launch_adj_finish(sim->p.prec, B, d_h0, d_theta, sim->p.theta0, sim->kconst, d_grad_h0,
                                           d_grad_theta, (hipStream_t)stream));
}

}  // extern "C"
