// Reverse mode of the thin-film lattice Boltzmann step: the hand-written
// vector-Jacobian product of one step of eq. "LBE" (arXiv:1810.07642, Sec. II)
// with respect to the pre-collision populations and the kappa field.
//
// Notation.  Forward step t, at every site x (pre-collision state f):
//   h = sum_l f_l, j = sum_l c_l f_l, u = j/h
//   p = -gamma (L h + kappa phi(h)),  phi(h) = (h_*/h)^n - (h_*/h)^m
//   G = grad_s p (isotropic gradient),  F = -h G - nu alpha(h) u + h a
//   f*_l = f_l + omega (feq_l(h, u) - f_l) + 3 w_l c_l . F,   f_l(x + c_l, t + 1) = f*_l(x).
// Adjoint.  lambda^t_l(x) = dLoss/df^t_l(x).  A reverse step at site x reads
// mu_l(x) = lambda^{t+1}_l(x + c_l) = dLoss/df*_l(x) and computes, at every
// site:
//   Lambda_F = 3 sum_l w_l c_l mu_l                       (from the source term)
//   lambda_G = -h Lambda_F                                (from F = -h G)
//   lambda_p = -div_s lambda_G                            (grad_s^T = -div_s)
//   lambda_u = omega sum_l mu_l dfeq_l/du - nu alpha Lambda_F
//   lambda_h = omega sum_l mu_l dfeq_l/dh + Lambda_F.(-G - nu alpha'(h) u + a)
//              - gamma L(lambda_p) - gamma kappa phi'(h) lambda_p - lambda_u.u/h    (L^T = L)
//   lambda_j = lambda_u / h
//   lambda^t_l = (1 - omega) mu_l + lambda_h + c_l . lambda_j
//   g_kappa += -gamma phi(h) lambda_p          (FP64 accumulation)
// and stores lambda^t_l(x) for step t-1 (layout: AdjRec).
// The forward moments h, j of step t come from the capture written by the
// forward step; the film pressure and its gradient are recomputed from h.
#include <algorithm>
#include <cstring>

#include "device.h"
#include "launch.h"
#include "sim.h"

namespace tflbm {

// Adjoint state layout ("push in y, pull in x", as the forward records).
// Records of kAdjW consecutive columns of one row, [ny][nstrips][RB]: the
// nine segments of kAdjW values ordered by c_ly (kSlot), the record padded to
// an odd number of 128-byte lines.  Entry l at (column X, row Y) holds
// nu_l(X, Y) = lambda_l(X, Y + c_ly): a site stores its adjoint populations
// at its own column, in the rows they are read from, so each strip writes
// whole records of its own; the lane of column x takes
// mu_l(x, y) = lambda_l(x + c_l) = nu_l(x + c_lx, y) from column x + c_lx
// of row y.  dLoss/dkappa is FP64 in records of 64 values [ny][nstrips][64]:
// the kAdjW columns and ten padding values, which the strip's halo lanes
// write, so that the record is four whole lines.
constexpr int kAdjW = 54;     // columns per strip and record
constexpr int kAdjHalo = 5;   // halo columns per side: two per reverse step and the shift between two steps
constexpr int kGkRB = 64 * 8;  // bytes of a dLoss/dkappa record
constexpr int kDropOffset = kDropBytes;  // a buffer offset past every row: the access is dropped
static_assert(kAdjW + 2 * kAdjHalo == 64, "a strip and its halo fill one wavefront");
template <typename T> struct AdjRec {
  static constexpr int SEG = kAdjW * (int)sizeof(T);
  static constexpr int LINES = (9 * SEG + 127) / 128;
  static constexpr int RB = (LINES % 2 ? LINES : LINES + 1) * 128;
  __host__ __device__ static constexpr int seg(int l) { return kSlot[l] * SEG; }
};

// With omega = 1 the step's adjoint is lambda^t_l = lambda_h + c_l . lambda_j
// (lam_of): three fields per site carry it between steps instead of nine
// populations.  They are stored at the site itself in records of 64 slots per
// field, [ny][nstrips][3][64] (lambda_h, lambda_jx, lambda_jy): the strip's
// kAdjW columns in slots 0 .. kAdjW-1 and ten padding slots that the halo
// lanes write, so a strip writes whole lines; the reverse step at (x, y)
// forms mu_l(x, y) = lambda_l(x + c_l) from the fields at column x + c_lx of
// row y + c_ly.
template <typename T> struct AdjRec1 {
  static constexpr int SEG = 64 * (int)sizeof(T);
  static constexpr int RB = 3 * SEG;
};

struct AdjArgs {
  const char *src;     // adjoint records at the end of step t (AdjRec; AdjRec1 with omega = 1)
  char *dst;           // adjoint records at the end of step t-1
  const char *cap;     // h, jx, jy of step t: capture records of the forward form
  const char *cap2;    // the same for step t-1 (two-step pass only)
  const void *kfield;  // kappa [ny][ldx] in T or nullptr
  char *gk;            // dLoss/dkappa records [ny][nstrips][64] FP64
  int nx, ny, ldx;
  int cnblk;           // capture records per row (those of the forward step)
  int capB, capRB;     // sites and bytes per capture record (the forward form's)
  int nstrips, H, ntiles, per_xcd;
  int n_exp, m_exp;
  double omega, gamma, nu, hstar, delta, ax, ay, g, kappa0;
};

int adj_record_columns() { return kAdjW; }
int adj_record_bytes_max(int prec) {
  const int a = prec == kF64 ? std::max(AdjRec<double>::RB, AdjRec1<double>::RB)
                             : std::max(AdjRec<float>::RB, AdjRec1<float>::RB);
  return std::max(a, kGkRB);
}

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

// Scalar coefficients of the reverse step in the working type.
template <typename T> struct AdjCoef {
  T omega, om1, gamma, nu, hstar, delta, three_d2, ax, ay, g, kap0, cA, cD;
  int n_exp, m_exp;
  __device__ explicit AdjCoef(const AdjArgs &A)
      : omega((T)A.omega), om1(T(1) - (T)A.omega), gamma((T)A.gamma), nu((T)A.nu), hstar((T)A.hstar),
        delta((T)A.delta), three_d2(T(3) * (T)A.delta * (T)A.delta), ax((T)A.ax), ay((T)A.ay), g((T)A.g),
        kap0((T)A.kappa0), cA((T)(3.0 * kW[1])), cD((T)(3.0 * kW[2])), n_exp(A.n_exp), m_exp(A.m_exp) {}
};

// Byte offsets of a lane inside one row of each array.  Rows are addressed
// through a wave-uniform buffer resource, so the marching loop spends no
// vector instructions on addresses.  Lane i of the strip starting at column
// x0 holds column a = x0 - kAdjHalo + i (periodic).
template <typename T> struct AdjLane {
  int nu[3];  // adjoint entry of columns a - 1, a, a + 1 (by c_lx + 1)
  int st;     // the lane's entry in its strip's record; kDropOffset for the halo lanes
  int nu1[3];  // omega = 1: field entry of columns a - 1, a, a + 1 (AdjRec1)
  int st1;     // omega = 1: the lane's slot in its strip's record (the halo lanes: padding)
  int cap;    // capture entry of column a
  int kap;    // kappa entry of column a
  int gk;     // dLoss/dkappa entry (the halo lanes: the record's padding)
  bool out;   // the lane's column belongs to the strip
  __device__ AdjLane(const AdjArgs &A, int strip, int lane) {
    const int x0 = strip * kAdjW, a = x0 - kAdjHalo + lane;
    const int xend = min(x0 + kAdjW, A.nx);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int col = wrap(a + c - 1, A.nx);
      const int s = col / kAdjW;
      nu[c] = s * AdjRec<T>::RB + (col - s * kAdjW) * (int)sizeof(T);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int col = wrap(a + c - 1, A.nx);
      const int s = col / kAdjW;
      nu1[c] = s * AdjRec1<T>::RB + (col - s * kAdjW) * (int)sizeof(T);
    }
    out = a >= x0 && a < xend;
    st = out ? strip * AdjRec<T>::RB + (a - x0) * (int)sizeof(T) : kDropOffset;
    st1 = strip * AdjRec1<T>::RB + ((lane - kAdjHalo) & 63) * (int)sizeof(T);
    const int col = wrap(a, A.nx);
    const int cb = col / A.capB;
    cap = cb * A.capRB + (col - cb * A.capB) * (int)sizeof(T);
    kap = col * (int)sizeof(T);
    gk = strip * kGkRB + ((lane - kAdjHalo) & 63) * 8;
  }
};

// lambda_l = lambda_h + c_l . lambda_j: the part of the step's adjoint that
// does not depend on mu (the whole of it when omega = 1).
template <typename T> __device__ __forceinline__ T lam_of(int l, T lh, T ljx, T ljy) {
  const int cx = kCx[l], cy = kCy[l];
  const T cl = cx == 0 ? (cy == 0 ? T(0) : (cy > 0 ? ljy : -ljy))
                       : (cy == 0 ? (cx > 0 ? ljx : -ljx)
                                  : (cx > 0 ? (cy > 0 ? ljx + ljy : ljx - ljy) : (cy > 0 ? ljy - ljx : -ljx - ljy)));
  return lh + cl;
}

// One input row of a reverse stage: the adjoint read (mu) and the forward
// moments and kappa of the same row.
template <typename T> struct AdjIn {
  T mu[9];
  T h, jx, jy, kap;
};
template <typename T> struct AdjCap {
  T h, jx, jy;
};

template <typename T> __device__ __forceinline__ T ld_t(rsrc_t r, int off);
template <> __device__ __forceinline__ float ld_t<float>(rsrc_t r, int off) { return ld_f32(r, off); }
template <> __device__ __forceinline__ double ld_t<double>(rsrc_t r, int off) { return ld_f64(r, off); }

// Row sizes in bytes.
template <typename T> __device__ __forceinline__ uint32_t adj_row_bytes(const AdjArgs &A) {
  return (uint32_t)A.nstrips * AdjRec<T>::RB;
}
__device__ __forceinline__ uint32_t cap_row_bytes(const AdjArgs &A) { return (uint32_t)A.cnblk * A.capRB; }

// mu_l of a row: nu_l(x + c_lx, row) from the adjoint records.
template <typename T>
__device__ __forceinline__ void load_mu(const AdjArgs &A, const AdjLane<T> &L, int row, T (&mu)[9]) {
  const uint32_t rb = adj_row_bytes<T>(A);
  const rsrc_t r = make_rsrc(A.src + (size_t)row * rb, rb);
#pragma unroll
  for (int l = 0; l < 9; ++l) mu[l] = ld_t<T>(r, L.nu[kCx[l] + 1] + AdjRec<T>::seg(l));
}

// omega = 1: lambda_h, lambda_jx, lambda_jy of a row at the columns x - 1,
// x, x + 1, as v[3 f + c] (f: the field, c = c_lx + 1).
template <typename T>
__device__ __forceinline__ void load_fields(const AdjArgs &A, const AdjLane<T> &L, int row, T (&v)[9]) {
  const uint32_t rb = (uint32_t)A.nstrips * AdjRec1<T>::RB;
  const rsrc_t r = make_rsrc(A.src + (size_t)row * rb, rb);
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[3 * f + c] = ld_t<T>(r, L.nu1[c] + f * AdjRec1<T>::SEG);
}

// omega = 1: mu of consecutive rows from the fields of the rows around them.
// The fields of row q give mu_l of row q - c_ly for every l; feeding row q
// completes mu of row q - 1 (its c_ly = +1 values come last) and leaves the
// parts of rows q and q + 1.
template <typename T> struct MuFromFields {
  T mc[3] = {0, 0, 0};  // mu_6, mu_7, mu_8 (c_ly = -1) of row q, from row q - 1
  T zc[3] = {0, 0, 0};  // mu_0, mu_1, mu_5 (c_ly = 0) of row q
  T mn[3] = {0, 0, 0};  // mu_6, mu_7, mu_8 of row q + 1, from row q
  __device__ __forceinline__ void feed(const T (&v)[9], T (&mu)[9]) {
    auto at = [&](int l) {
      const int c = kCx[l] + 1;
      return lam_of(l, v[c], v[3 + c], v[6 + c]);
    };
    mu[2] = at(2);
    mu[3] = at(3);
    mu[4] = at(4);
    mu[0] = zc[0];
    mu[1] = zc[1];
    mu[5] = zc[2];
    mu[6] = mc[0];
    mu[7] = mc[1];
    mu[8] = mc[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) mc[i] = mn[i];
    zc[0] = at(0);
    zc[1] = at(1);
    zc[2] = at(5);
    mn[0] = at(6);
    mn[1] = at(7);
    mn[2] = at(8);
  }
};

// omega = 1: stores lambda_h, lambda_j of row y at the lane's slot.
template <typename T>
__device__ __forceinline__ void store_fields(const AdjArgs &A, const AdjLane<T> &L, int y, T lh, T ljx, T ljy) {
  const uint32_t rb = (uint32_t)A.nstrips * AdjRec1<T>::RB;
  const rsrc_t r = make_rsrc(A.dst + (size_t)y * rb, rb);
  st_t(r, L.st1, lh);
  st_t(r, L.st1 + AdjRec1<T>::SEG, ljx);
  st_t(r, L.st1 + 2 * AdjRec1<T>::SEG, ljy);
}

// h, j_x, j_y of a row from the capture records of a forward step.
template <typename T>
__device__ __forceinline__ void load_cap(const AdjArgs &A, const char *cap, const AdjLane<T> &L, int row, T &h, T &jx,
                                         T &jy) {
  const int SEG = A.capB * (int)sizeof(T);
  const uint32_t rb = cap_row_bytes(A);
  const rsrc_t r = make_rsrc(cap + (size_t)row * rb, rb);
  h = ld_t<T>(r, L.cap);
  jx = ld_t<T>(r, L.cap + SEG);
  jy = ld_t<T>(r, L.cap + 2 * SEG);
}

template <typename T>
__device__ __forceinline__ T load_kap(const AdjArgs &A, const AdjLane<T> &L, int row) {
  const uint32_t rb = (uint32_t)A.ldx * sizeof(T);
  return ld_t<T>(make_rsrc((const char *)A.kfield + (size_t)row * rb, rb), L.kap);
}

// The resource of row y of the dLoss/dkappa records; with `valid` false an
// empty range (its loads read zeros and touch no memory).
__device__ __forceinline__ rsrc_t gk_row(const AdjArgs &A, int y, bool valid = true) {
  const uint32_t rb = (uint32_t)A.nstrips * kGkRB;
  return make_rsrc(A.gk + (size_t)y * rb, valid ? rb : 0u);
}

// One reverse step as a machine over the rows of a strip, one column per
// lane.  Rows enter in increasing y.  Once row r has entered (`push`), the
// stage has formed the film pressure and lambda_p of row r-1, and `out` gives
// the adjoint populations of row r-2.  The x stencils read the neighbouring
// lanes, so the first and last two lanes of the strip are halo.  Row indices
// count from the newest: 0 = r, 1 = r-1, 2 = r-2, 3 = r-3.  Both x-stencils
// of a row are folded into two numbers per quantity at the row's entry
// (the difference and the weighted sum of its left and right neighbours), so
// that the rows kept in flight are single values.
template <typename T> struct AdjStage {
  T h0 = 0, h1 = 0, h2 = 0;                               // h
  T s0 = 0, s1 = 0, s2 = 0;                               // h(x-1) + h(x+1)
  T jx0 = 0, jx1 = 0, jx2 = 0, jy0 = 0, jy1 = 0, jy2 = 0;  // j
  T k0 = 0, k1 = 0, k2 = 0;                               // kappa
  T Fx0 = 0, Fx1 = 0, Fx2 = 0, Fy0 = 0, Fy1 = 0, Fy2 = 0;  // Lambda_F
  T ga0 = 0, ga1 = 0, ga2 = 0;   // lambda_Gx(x+1) - lambda_Gx(x-1)
  T gb0 = 0, gb1 = 0, gb2 = 0;   // cA lambda_Gy(x) + cD (lambda_Gy(x-1) + lambda_Gy(x+1))
  T pa1 = 0, pa2 = 0, pa3 = 0;   // p(x+1) - p(x-1)
  T pb1 = 0, pb2 = 0, pb3 = 0;   // cA p(x) + cD (p(x-1) + p(x+1))
  T q1 = 0, q2 = 0, q3 = 0;      // lambda_p
  T qs1 = 0, qs2 = 0, qs3 = 0;   // lambda_p(x-1) + lambda_p(x+1)
  T ih1 = 0, ih2 = 0, rn1 = 0, rn2 = 0, rm1 = 0, rm2 = 0;  // 1/h, (h_*/h)^n, (h_*/h)^m

  // Row r enters with its pre-shifted adjoint mu and the forward h, j and
  // kappa; `full` = rows r-1 and r-2 entered before it.
  __device__ __forceinline__ void push(const T (&mu)[9], T h, T jx, T jy, T kap, bool full, const AdjCoef<T> &C) {
    h2 = h1; h1 = h0; h0 = h;
    s2 = s1; s1 = s0; s0 = from_left(h) + from_right(h);
    jx2 = jx1; jx1 = jx0; jx0 = jx;
    jy2 = jy1; jy1 = jy0; jy0 = jy;
    k2 = k1; k1 = k0; k0 = kap;
    Fx2 = Fx1; Fx1 = Fx0;
    Fy2 = Fy1; Fy1 = Fy0;
    lambda_force(mu, C.cA, C.cD, Fx0, Fy0);
    // lambda_G = -h Lambda_F, kept as the two combinations its divergence reads
    const T gx = -h * Fx0, gy = -h * Fy0;
    ga2 = ga1; ga1 = ga0; ga0 = from_right(gx) - from_left(gx);
    gb2 = gb1; gb1 = gb0; gb0 = madd(C.cA, gy, C.cD * (from_left(gy) + from_right(gy)));
    if (!full) return;
    // forward film pressure of row r-1 (Laplacian over rows r-2 .. r)
    const T lap = (T(4) * ((s1 + h0) + h2) + (s0 + s2) - T(20) * h1) * T(1.0 / 6.0);
    ih2 = ih1; rn2 = rn1; rm2 = rm1;
    ih1 = recip(h1);
    powers(C.hstar * ih1, C.n_exp, C.m_exp, rn1, rm1);
    const T p = -C.gamma * (lap + k1 * (rn1 - rm1));
    pa3 = pa2; pa2 = pa1; pa1 = from_right(p) - from_left(p);
    pb3 = pb2; pb2 = pb1; pb1 = madd(C.cA, p, C.cD * (from_left(p) + from_right(p)));
    // lambda_p of row r-1 = -div_s lambda_G (lambda_G rows r-2 .. r)
    const T q = -(madd(C.cA, ga1, C.cD * (ga0 + ga2)) + (gb0 - gb2));
    q3 = q2; q2 = q1; q1 = q;
    qs3 = qs2; qs2 = qs1; qs1 = from_left(q) + from_right(q);
  }

  // Adjoint populations lambda^t_l of row r-2 from that row's mu, and the
  // row's term -gamma phi(h) lambda_p of dLoss/dkappa.
  __device__ __forceinline__ void out(const T (&mu)[9], T (&lam)[9], double &gterm, const AdjCoef<T> &C) const {
    T lh, ljx, ljy;
    out_moments(mu, lh, ljx, ljy, gterm, C);
#pragma unroll
    for (int l = 0; l < 9; ++l) lam[l] = madd(C.om1, mu[l], lam_of(l, lh, ljx, ljy));
  }

  // lambda_h and lambda_j of row r-2 (lambda^t_l = (1 - omega) mu_l +
  // lambda_h + c_l . lambda_j), and the row's term of dLoss/dkappa.
  __device__ __forceinline__ void out_moments(const T (&mu)[9], T &lh_out, T &ljx_out, T &ljy_out, double &gterm,
                                              const AdjCoef<T> &C) const {
    const T h = h2, inv_h = ih2;
    const T ux = jx2 * inv_h, uy = jy2 * inv_h;
    // forward pressure gradient (p rows r-3 .. r-1)
    const T Gx = madd(C.cA, pa2, C.cD * (pa1 + pa3));
    const T Gy = pb1 - pb3;
    // Laplacian of lambda_p (rows r-3 .. r-1)
    const T lapq = (T(4) * ((qs2 + q1) + q3) + (qs1 + qs3) - T(20) * q2) * T(1.0 / 6.0);
    const T lp = q2;

    const T invD = recip(madd(T(2) * h, h, madd(T(6) * C.delta, h, C.three_d2)));
    const T alpha = T(6) * h * invD;
    const T dalpha = T(6) * madd(T(-2) * h, h, C.three_d2) * (invD * invD);
    const T phi = rn2 - rm2;
    const T dphi = (T(C.m_exp) * rm2 - T(C.n_exp) * rn2) * inv_h;

    // omega sum_l mu_l dfeq_l/dh and omega sum_l mu_l dfeq_l/du over pairs
    // of opposite populations: S = mu_l + mu_-l takes the parts of the
    // derivatives even in c, D = mu_l - mu_-l the odd ones
    const T usq = madd(ux, ux, uy * uy);
    const T gh = C.g * h;
    const T up = ux + uy, um = uy - ux;
    const T S15 = mu[1] + mu[5], D15 = mu[1] - mu[5];
    const T S37 = mu[3] + mu[7], D37 = mu[3] - mu[7];
    const T S26 = mu[2] + mu[6], D26 = mu[2] - mu[6];
    const T S48 = mu[4] + mu[8], D48 = mu[4] - mu[8];
    // d/dh: rest 1 - 5gh/3 - 2u^2/3; axes gh/3 + cu/3 + cu^2/2 - u^2/6;
    // diagonals gh/12 + cu/12 + cu^2/8 - u^2/24
    T sh = mu[0] * madd(gh, T(-5.0 / 3.0), madd(usq, T(-2.0 / 3.0), T(1)));
    sh = madd(S15 + S37, madd(gh, T(1.0 / 3.0), usq * T(-1.0 / 6.0)), sh);
    sh = madd(T(0.5), madd(S15, ux * ux, S37 * (uy * uy)), sh);
    sh = madd(T(1.0 / 3.0), madd(D15, ux, D37 * uy), sh);
    sh = madd(S26 + S48, madd(gh, T(1.0 / 12.0), usq * T(-1.0 / 24.0)), sh);
    sh = madd(T(0.125), madd(S26, up * up, S48 * (um * um)), sh);
    sh = madd(T(1.0 / 12.0), madd(D26, up, D48 * um), sh);
    // d/du = h (c1 c + c2 (c.u) c - c3 u): rest -4u/3; axes (1/3, 1, 1/3);
    // diagonals (1/12, 1/4, 1/12)
    T sx = mu[0] * ux * T(-4.0 / 3.0);
    sx = madd(D15, T(1.0 / 3.0), sx);
    sx = madd(S15 - T(0.5) * S37, ux * T(2.0 / 3.0), sx);
    sx = madd(D26 - D48, T(1.0 / 12.0), sx);
    sx = madd(S26, madd(up, T(0.25), ux * T(-1.0 / 12.0)), sx);
    sx = madd(S48, madd(um, T(-0.25), ux * T(-1.0 / 12.0)), sx);
    T sy = mu[0] * uy * T(-4.0 / 3.0);
    sy = madd(D37, T(1.0 / 3.0), sy);
    sy = madd(S37 - T(0.5) * S15, uy * T(2.0 / 3.0), sy);
    sy = madd(D26 + D48, T(1.0 / 12.0), sy);
    sy = madd(S26, madd(up, T(0.25), uy * T(-1.0 / 12.0)), sy);
    sy = madd(S48, madd(um, T(0.25), uy * T(-1.0 / 12.0)), sy);
    const T fric = C.nu * alpha;
    const T lux = madd(C.omega * h, sx, -fric * Fx2);
    const T luy = madd(C.omega * h, sy, -fric * Fy2);
    T lh = C.omega * sh + Fx2 * (-Gx - C.nu * dalpha * ux + C.ax) + Fy2 * (-Gy - C.nu * dalpha * uy + C.ay) -
           C.gamma * lapq - C.gamma * k2 * dphi * lp;
    lh -= (lux * ux + luy * uy) * inv_h;
    lh_out = lh;
    ljx_out = lux * inv_h;
    ljy_out = luy * inv_h;
    gterm = -(double)C.gamma * (double)phi * (double)lp;
  }
};

// Stores lambda^t_l of row y: entry l of the lane's column goes to row
// y - c_ly, where the step before reads it.  The halo lanes' stores are
// dropped (kDropOffset), so a strip writes the contiguous entries of its
// own records.
template <typename T>
__device__ __forceinline__ void store_lambda(const AdjArgs &A, const AdjLane<T> &L, int y, const T (&lam)[9]) {
  const uint32_t rb = adj_row_bytes<T>(A);
  const int yN = (y + 1 == A.ny) ? 0 : y + 1;
  const int yS = (y == 0) ? A.ny - 1 : y - 1;
  // by c_ly + 1: c_ly = -1 -> row y + 1, 0 -> row y, +1 -> row y - 1
  const rsrc_t rd[3] = {make_rsrc(A.dst + (size_t)yN * rb, rb), make_rsrc(A.dst + (size_t)y * rb, rb),
                        make_rsrc(A.dst + (size_t)yS * rb, rb)};
#pragma unroll
  for (int l = 0; l < 9; ++l) st_t(rd[kCy[l] + 1], L.st + AdjRec<T>::seg(l), lam[l]);
}

// One reverse step.  A workgroup is one wavefront marching up a strip of
// kAdjW columns (plus kAdjHalo halo columns per side, of which the stencils
// of one step need two) over a chunk of rows; it reads rows y0-2 .. yend+1
// (W1: the fields of rows y0-3 .. yend+2) and writes rows y0 .. yend-1.
template <typename T, bool KF, bool W1 = false>
__global__ __launch_bounds__(64) void adj_step_kernel(AdjArgs A) {
  const int b = blockIdx.x;
  const int tile = (b & 7) * A.per_xcd + (b >> 3);
  if (tile >= A.ntiles) return;
  const int strip = tile % A.nstrips;
  const int chunk = tile / A.nstrips;
  const int y0 = chunk * A.H;
  const int yend = min(y0 + A.H, A.ny);
  const int ny = A.ny;
  const AdjLane<T> L(A, strip, threadIdx.x);

  const AdjCoef<T> C(A);
  AdjStage<T> S;
  T mu1[9], mu2[9], mun[9];
  T hn, jxn, jyn, kn = C.kap0;
#pragma unroll
  for (int l = 0; l < 9; ++l) mu1[l] = mu2[l] = 0;

  const int K = (yend - y0) + 4;
  int ry = wrap(y0 - 2, ny);
  // W1: mu of row r needs the fields of rows r-1 .. r+1; they are read one
  // row ahead and fed into `mf`, which completes mu of the row before
  MuFromFields<T> mf;
  auto load_row = [&](int row) {
    if constexpr (W1) load_fields(A, L, row + 1 == ny ? 0 : row + 1, mun);
    else load_mu(A, L, row, mun);
    load_cap(A, A.cap, L, row, hn, jxn, jyn);
    if constexpr (KF) kn = load_kap(A, L, row);
  };
  if constexpr (W1) {
    T v[9], unused[9];
    load_fields(A, L, wrap(y0 - 3, ny), v);
    mf.feed(v, unused);
    load_fields(A, L, ry, v);
    mf.feed(v, unused);
  }
  load_row(ry);
  // dLoss/dkappa of the next output row, in two slots taken by the parity of
  // the row in the unrolled loop (gcur: this row's entry, gnext: where the
  // next row's goes), so that the value never moves between registers: a
  // move would wait for the load just issued
  double gka = ld_f64(gk_row(A, y0), L.gk), gkb = 0.0;

  auto iteration = [&](int k, double &gcur, double &gnext) {
    T mu0[9];
    if constexpr (W1) {
      mf.feed(mun, mu0);
    } else {
#pragma unroll
      for (int l = 0; l < 9; ++l) mu0[l] = mun[l];
    }
    const T h = hn, jx = jxn, jy = jyn, kap = kn;
    const int rn = (ry + 1 == ny) ? 0 : ry + 1;
    if (k + 1 < K) load_row(rn);
    S.push(mu0, h, jx, jy, kap, k >= 2, C);
    if (k >= 4) {
      // output row y = r-2
      const int y = y0 + (k - 4);
      double gt;
      if constexpr (W1) {
        T lh, ljx, ljy;
        S.out_moments(mu2, lh, ljx, ljy, gt, C);
        store_fields(A, L, y, lh, ljx, ljy);
      } else {
        T lam[9];
        S.out(mu2, lam, gt, C);
        store_lambda(A, L, y, lam);
      }
      // the next row's entry is read one row ahead, on every row (past the
      // last an empty range): a load skipped on some path would make the
      // compiler join its two values right after it, waiting for the load and
      // for everything issued before it
      double g = gcur;
      gnext = ld_f64(gk_row(A, y + 1, k + 1 < K), L.gk);
      if (L.out) g += gt;
      st_f64(gk_row(A, y), L.gk, g);
    }
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      mu2[l] = mu1[l];
      mu1[l] = mu0[l];
    }
    ry = rn;
  };
  // FP32 with omega = 1: rows in groups of six, as in adj_step2_kernel (three
  // wavefronts per SIMD either way); elsewhere the unrolled loop would cost a
  // wavefront per SIMD (FP64 one-step passes reach 256 VGPRs and one)
  int k = 0;
  if constexpr (W1 && sizeof(T) == 4) {
    for (; k + 5 < K; k += 6) {
      iteration(k, gka, gkb);
      iteration(k + 1, gkb, gka);
      iteration(k + 2, gka, gkb);
      iteration(k + 3, gkb, gka);
      iteration(k + 4, gka, gkb);
      iteration(k + 5, gkb, gka);
    }
  }
  // one slot (the entry is copied before the next one is loaded); k is even
  // here, so gka holds the next output row's entry
  for (; k < K; ++k) iteration(k, gka, gka);
}

// Two reverse steps, t and t-1, in one pass.  The step-t stage runs as in
// adj_step_kernel, five rows ahead of the step-(t-1) stage, and hands it its
// adjoint through a ring of five rows in LDS: the step-(t-1) input
// mu_l(x, y) = lambda^t_l(x + c_l, y + c_l) is read from the ring rather
// than stored to memory and streamed back.  The step-t contribution to
// dLoss/dkappa waits in a second ring until the step-(t-1) stage reaches the
// same row, so that g_kappa is read and written once per pass and receives
// the two terms in the order of two single steps.  The workgroup is a single
// wavefront, so the ring needs no barrier between wavefronts.  Strips are
// kAdjW columns plus five halo columns per side (two per stage plus the
// one-column shift between them); rows y0-5 .. yend+4 are read (W1: the
// fields of rows y0-6 .. yend+5).
template <typename T, bool KF, bool W1 = false, bool LONG = false>
__global__ __launch_bounds__(64) void adj_step2_kernel(AdjArgs A) {
  __shared__ T ring[5][9][64];
  __shared__ double gring[4][64];
  const int b = blockIdx.x;
  const int tile = (b & 7) * A.per_xcd + (b >> 3);
  if (tile >= A.ntiles) return;
  const int strip = tile % A.nstrips;
  const int chunk = tile / A.nstrips;
  const int y0 = chunk * A.H;
  const int yend = min(y0 + A.H, A.ny);
  const int lane = threadIdx.x;
  const int ny = A.ny;
  const AdjLane<T> L(A, strip, lane);
  // ring columns of x - 1 and x + 1 (the end lanes read themselves: halo)
  const int lw = lane > 0 ? lane - 1 : 0, le = lane < 63 ? lane + 1 : 63;

  const AdjCoef<T> C(A);
  AdjStage<T> S1, S2;
  T mu1[9], mu2[9];
  // kappa of the step-t input rows of the last three iterations: the
  // step-(t-1) stage takes each row three iterations later
  T kd1 = C.kap0, kd2 = C.kap0, kd3 = C.kap0;
#pragma unroll
  for (int l = 0; l < 9; ++l) mu1[l] = mu2[l] = 0;

  // iteration k: step-t input row y0-5+k, step-t output row y0-7+k (k >= 4),
  // step-(t-1) input row y0-8+k (k >= 6), step-(t-1) output row y0-10+k (k >= 10).
  // Input rows are loaded two iterations ahead, into the buffers the
  // iteration two back consumed (ia/ca for even k, ib/cb for odd k).
  const int K = (yend - y0) + 10;
  AdjIn<T> ia, ib;
  AdjCap<T> ca = {}, cb = {};
  // W1: mu of row r needs the fields of rows r-1 .. r+1; they are read one
  // row ahead (into in.mu) and fed into `mf`, which completes mu of the row
  // before
  MuFromFields<T> mf;
  auto load1 = [&](int k, AdjIn<T> &in) {
    const int row = wrap(y0 - 5 + k, ny);
    if constexpr (W1) load_fields(A, L, row + 1 == ny ? 0 : row + 1, in.mu);
    else load_mu(A, L, row, in.mu);
    load_cap(A, A.cap, L, row, in.h, in.jx, in.jy);
    in.kap = C.kap0;
    if constexpr (KF) in.kap = load_kap(A, L, row);
  };
  if constexpr (W1) {
    T v[9], unused[9];
    load_fields(A, L, wrap(y0 - 6, ny), v);
    mf.feed(v, unused);
    load_fields(A, L, wrap(y0 - 5, ny), v);
    mf.feed(v, unused);
  }
  load1(0, ia);
  load1(1, ib);
  // dLoss/dkappa of the next output row, in two slots taken by the parity of
  // the row, as in adj_step_kernel
  double gka = ld_f64(gk_row(A, y0), L.gk), gkb = 0.0;

  auto iteration = [&](int k, AdjIn<T> &in, AdjCap<T> &cin, double &gcur, double &gnext) {
    T mu0[9];
    if constexpr (W1) {
      mf.feed(in.mu, mu0);
    } else {
#pragma unroll
      for (int l = 0; l < 9; ++l) mu0[l] = in.mu[l];
    }
    const T h = in.h, jx = in.jx, jy = in.jy, kap = in.kap;
    const T h_2 = cin.h, jx_2 = cin.jx, jy_2 = cin.jy, kap_2 = kd3;
    kd3 = kd2;
    kd2 = kd1;
    kd1 = kap;
    if (k + 2 < K) load1(k + 2, in);
    if (k + 2 >= 6 && k + 2 < K) load_cap(A, A.cap2, L, wrap(y0 - 6 + k, ny), cin.h, cin.jx, cin.jy);

    S1.push(mu0, h, jx, jy, kap, k >= 2, C);
    if (k >= 4) {
      T lam[9];
      double gt;
      if constexpr (W1) {
        T lh, ljx, ljy;
        S1.out_moments(mu2, lh, ljx, ljy, gt, C);
#pragma unroll
        for (int l = 0; l < 9; ++l) lam[l] = lam_of(l, lh, ljx, ljy);
      } else {
        S1.out(mu2, lam, gt, C);
      }
      const int s = k % 5;
#pragma unroll
      for (int l = 0; l < 9; ++l) ring[s][l][lane] = lam[l];
      gring[k & 3][lane] = gt;
    }
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      mu2[l] = mu1[l];
      mu1[l] = mu0[l];
    }

    if (k >= 6) {
      __syncthreads();
      // step-(t-1) input row y' = y0-8+k: lambda^t rows y'-1 .. y'+1 were
      // written at iterations k-2 .. k
      T m[9];
#pragma unroll
      for (int l = 0; l < 9; ++l)
        m[l] = ring[(k - 1 + kCy[l]) % 5][l][kCx[l] == 0 ? lane : (kCx[l] > 0 ? le : lw)];
      S2.push(m, h_2, jx_2, jy_2, kap_2, k >= 8, C);
      if (k >= 10) {
        // output row y = y' - 2; its mu from lambda^t rows y-1 .. y+1
        const int y = y0 + (k - 10);
        T mo[9];
#pragma unroll
        for (int l = 0; l < 9; ++l)
          mo[l] = ring[(k - 3 + kCy[l]) % 5][l][kCx[l] == 0 ? lane : (kCx[l] > 0 ? le : lw)];
        double gt;
        if constexpr (W1) {
          T lh, ljx, ljy;
          S2.out_moments(mo, lh, ljx, ljy, gt, C);
          store_fields(A, L, y, lh, ljx, ljy);
        } else {
          T lam[9];
          S2.out(mo, lam, gt, C);
          store_lambda(A, L, y, lam);
        }
        double g = gcur;  // the next row's entry is read on every row, as in adj_step_kernel
        gnext = ld_f64(gk_row(A, y + 1, k + 1 < K), L.gk);
        if (L.out) {
          g += gring[(k + 1) & 3][lane];  // the step-t term of row y, from iteration k-3
          g += gt;
        }
        st_f64(gk_row(A, y), L.gk, g);
      }
    }
  };
  // rows in groups of six, a whole number of turns of every row history
  // (three rows) and of the two input buffers, so that the compiler can keep
  // each history value in place instead of moving it along every row (a
  // quarter of the loop's VALU instructions were such moves with pairs):
  // 4096^2 FP32 with omega = 1 186 -> 174 us per step, 1024^2 20.0 -> 17.7
  // LONG (chunks of at least kAdjLongRows rows): the ten rows before the first
  // output row, then groups in which the compiler is told that every row
  // outputs and loads two rows ahead, so a group is straight-line code whose
  // waits leave the younger loads and stores in flight (4096^2 FP32 157.9 ->
  // 149.0 us per step, bitwise the same); on short chunks, where most rows
  // fall outside such groups, this loses (1024^2 16.5 -> 17.5 us) and the
  // kernel keeps the plain groups
  int k = 0;
  if constexpr (LONG) {
    for (; k < 10; k += 2) {  // K > 10: a chunk has at least one row
      iteration(k, ia, ca, gka, gkb);
      iteration(k + 1, ib, cb, gkb, gka);
    }
    for (; k + 7 < K; k += 6) {
      // k is the same in every lane.  Stated here, before the range, it keeps
      // the row arithmetic and the buffer resources scalar in the rows after
      // the groups too: without it the compiler took k as per-lane in the
      // two-row loop below and wrapped each of its row loads and stores in a
      // loop over the lanes' resources (four readfirstlanes, two 64-bit
      // compares and an exec-mask branch each; 1 % of the VALU instructions
      // at 4096^2, no change in time).  Stated inside `iteration` instead, it
      // hides the range from the stage tests, which then branch
      // (4096^2 149 -> 166 us per step).
      k = __builtin_amdgcn_readfirstlane(k);
      __builtin_assume(k >= 10 && k + 7 < K);
      iteration(k, ia, ca, gka, gkb);
      iteration(k + 1, ib, cb, gkb, gka);
      iteration(k + 2, ia, ca, gka, gkb);
      iteration(k + 3, ib, cb, gkb, gka);
      iteration(k + 4, ia, ca, gka, gkb);
      iteration(k + 5, ib, cb, gkb, gka);
    }
  } else {
    for (; k + 5 < K; k += 6) {
      iteration(k, ia, ca, gka, gkb);
      iteration(k + 1, ib, cb, gkb, gka);
      iteration(k + 2, ia, ca, gka, gkb);
      iteration(k + 3, ib, cb, gkb, gka);
      iteration(k + 4, ia, ca, gka, gkb);
      iteration(k + 5, ib, cb, gkb, gka);
    }
  }
  for (; k + 1 < K; k += 2) {
    iteration(k, ia, ca, gka, gkb);
    iteration(k + 1, ib, cb, gkb, gka);
  }
  if (k < K) iteration(k, ia, ca, gka, gkb);
}

// nu_l(x, y) = lambda^N_l(x, y + c_ly) = dLoss/dh_N(x, y + c_ly) for every l
// (h_N = sum_l f_l); dLoss/dkappa = 0, its padding included.  Thread i of a
// row: entry i of the row's dLoss/dkappa records, and column i if i < nx.
// W1: lambda_h = dLoss/dh_N, lambda_j = 0 (so lambda_l = dLoss/dh_N for
// every l); thread i writes slot i of the row's field records, padding
// included.
template <typename T, bool W1 = false>
__global__ void adj_seed_kernel(AdjArgs A, const double *grad_h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (i >= A.nstrips * 64) return;
  ((double *)(A.gk + (size_t)y * A.nstrips * kGkRB))[i] = 0.0;
  if constexpr (W1) {
    const int s = i / 64, slot = i - 64 * s, x = s * kAdjW + slot;
    T *rec = (T *)(A.dst + ((size_t)y * A.nstrips + s) * AdjRec1<T>::RB);
    rec[slot] = slot < kAdjW && x < A.nx ? (T)grad_h[(size_t)y * A.nx + x] : T(0);
    rec[64 + slot] = T(0);
    rec[128 + slot] = T(0);
    return;
  }
  if (i >= A.nx) return;
  const int s = i / kAdjW;
  char *ent = A.dst + ((size_t)y * A.nstrips + s) * AdjRec<T>::RB + (size_t)(i - s * kAdjW) * sizeof(T);
  for (int l = 0; l < 9; ++l) {
    const int ys = wrap(y + kCy[l], A.ny);
    *(T *)(ent + AdjRec<T>::seg(l)) = (T)grad_h[(size_t)ys * A.nx + i];
  }
}

// dLoss/dh0 = sum_l lambda^0_l dE_l/dh0 with lambda^0_l(x, y) = nu_l(x, y - c_ly)
// (W1: lam_of the fields at (x, y));
// dLoss/dtheta = dLoss/dkappa * (n-1)(m-1)/((n-m) h_*) * sin(theta).
template <typename T, bool W1 = false>
__global__ void adj_finish_kernel(AdjArgs A, const double *h0, const double *theta, double theta0, double kconst,
                                  double *grad_h0, double *grad_theta) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.nx) return;
  const size_t od = (size_t)y * A.nx + x;
  const int st = x / kAdjW, pos = x - st * kAdjW;
  if (grad_h0) {
    const double h = h0[od];
    const size_t ent = (size_t)st * AdjRec<T>::RB + (size_t)pos * sizeof(T);
    T fh = 0, fx = 0, fy = 0;
    if constexpr (W1) {
      const T *rec = (const T *)(A.src + ((size_t)y * A.nstrips + st) * AdjRec1<T>::RB);
      fh = rec[pos];
      fx = rec[64 + pos];
      fy = rec[128 + pos];
    }
    double s = 0.0;
    for (int l = 0; l < 9; ++l) {
      const int ys = wrap(y - kCy[l], A.ny);
      const double lam = W1 ? (double)lam_of(l, fh, fx, fy)
                            : (double)*(const T *)(A.src + (size_t)ys * A.nstrips * AdjRec<T>::RB + ent + AdjRec<T>::seg(l));
      const double dE = l == 0 ? 1.0 - A.g * h * (5.0 / 3.0) : ((l & 1) ? A.g * h / 3.0 : A.g * h / 12.0);
      s += lam * dE;
    }
    grad_h0[od] = s;
  }
  if (grad_theta) {
    const double th = theta ? theta[od] : theta0;
    const double gk = ((const double *)(A.gk + ((size_t)y * A.nstrips + st) * kGkRB))[pos];
    grad_theta[od] = gk * kconst * sin(th);
  }
}

// Chunks from which the two-step reverse kernel takes its LONG row loop.
constexpr int kAdjLongRows = 32;

template <typename T, bool W1>
static hipError_t adj_step_t(const AdjArgs &B, bool kf, int ns, hipStream_t s) {
  const dim3 grid(8 * B.per_xcd), block(64);
  if (ns == 2) {
    const bool lng = B.H >= kAdjLongRows;
    if (kf) {
      if (lng) adj_step2_kernel<T, true, W1, true><<<grid, block, 0, s>>>(B);
      else adj_step2_kernel<T, true, W1><<<grid, block, 0, s>>>(B);
    } else {
      if (lng) adj_step2_kernel<T, false, W1, true><<<grid, block, 0, s>>>(B);
      else adj_step2_kernel<T, false, W1><<<grid, block, 0, s>>>(B);
    }
  } else {
    if (kf) adj_step_kernel<T, true, W1><<<grid, block, 0, s>>>(B);
    else adj_step_kernel<T, false, W1><<<grid, block, 0, s>>>(B);
  }
  return hipGetLastError();
}

hipError_t launch_adj_step(int prec, const AdjArgs &B, bool kf, int ns, bool w1, hipStream_t s) {
  if (prec == kF64) return w1 ? adj_step_t<double, true>(B, kf, ns, s) : adj_step_t<double, false>(B, kf, ns, s);
  return w1 ? adj_step_t<float, true>(B, kf, ns, s) : adj_step_t<float, false>(B, kf, ns, s);
}

template <typename T, bool W1>
static int adj_occupancy_t(bool kf, int ns) {
  int n = 0;
  hipError_t e;
  if (ns == 2)
    e = kf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj_step2_kernel<T, true, W1>, 64, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj_step2_kernel<T, false, W1>, 64, 0);
  else
    e = kf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj_step_kernel<T, true, W1>, 64, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adj_step_kernel<T, false, W1>, 64, 0);
  return e == hipSuccess ? n : 0;
}

int adj_blocks_per_cu(int prec, bool kf, int ns, bool w1) {
  if (prec == kF64) return w1 ? adj_occupancy_t<double, true>(kf, ns) : adj_occupancy_t<double, false>(kf, ns);
  return w1 ? adj_occupancy_t<float, true>(kf, ns) : adj_occupancy_t<float, false>(kf, ns);
}

hipError_t launch_adj_seed(int prec, const AdjArgs &B, const double *grad_h, bool w1, hipStream_t s) {
  const dim3 block(256), grid((B.nstrips * 64 + 255) / 256, B.ny);
  if (prec == kF64) {
    if (w1) adj_seed_kernel<double, true><<<grid, block, 0, s>>>(B, grad_h);
    else adj_seed_kernel<double, false><<<grid, block, 0, s>>>(B, grad_h);
  } else {
    if (w1) adj_seed_kernel<float, true><<<grid, block, 0, s>>>(B, grad_h);
    else adj_seed_kernel<float, false><<<grid, block, 0, s>>>(B, grad_h);
  }
  return hipGetLastError();
}

hipError_t launch_adj_finish(int prec, const AdjArgs &B, const double *h0, const double *theta, double theta0,
                             double kconst, double *grad_h0, double *grad_theta, bool w1, hipStream_t s) {
  const dim3 block(256), grid((B.nx + 255) / 256, B.ny);
  if (prec == kF64) {
    if (w1) adj_finish_kernel<double, true><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
    else adj_finish_kernel<double, false><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
  } else {
    if (w1) adj_finish_kernel<float, true><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
    else adj_finish_kernel<float, false><<<grid, block, 0, s>>>(B, h0, theta, theta0, kconst, grad_h0, grad_theta);
  }
  return hipGetLastError();
}

static size_t adj_buf_bytes(const tflbm_sim *s) {
  const size_t rb = s->w1 ? (s->p.prec == kF64 ? AdjRec1<double>::RB : AdjRec1<float>::RB)
                          : (s->p.prec == kF64 ? AdjRec<double>::RB : AdjRec<float>::RB);
  return (size_t)s->p.ny * s->adj_nstrips * rb;
}
static size_t gk_bytes(const tflbm_sim *s) { return (size_t)s->p.ny * s->adj_nstrips * kGkRB; }
static size_t round4k(size_t v) { return (v + 4095) / 4096 * 4096; }

// AdjArgs of the current adjoint buffers, shaped for `ns` steps per pass.
static AdjArgs make_adj_args(const tflbm_sim *s, void *d_adj, int ns = 1) {
  AdjArgs B;
  std::memset(&B, 0, sizeof(B));
  char *base = (char *)d_adj;
  const size_t nb = round4k(adj_buf_bytes(s));
  B.src = base + (s->adj_cur == 0 ? 0 : nb);
  B.dst = base + (s->adj_cur == 0 ? nb : 0);
  B.gk = base + 2 * nb;
  B.kfield = s->kfield == kKappa ? (const void *)(s->ws + s->off_k) : nullptr;
  B.nx = s->p.nx;
  B.ny = s->p.ny;
  B.ldx = s->ldx;
  B.cnblk = s->nblk;
  B.capB = record_sites(s->p.prec);
  B.capRB = capture_record_bytes(s->p.prec);
  B.nstrips = s->adj_nstrips;  // the record columns of the adjoint state; both kernels march them
  B.H = ns == 2 ? s->adj2_rows : s->adj_rows;
  B.ntiles = ns == 2 ? s->adj2_ntiles : s->adj_ntiles;
  B.per_xcd = ns == 2 ? s->adj2_per_xcd : s->adj_per_xcd;
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
  return 2 * round4k(adj_buf_bytes(sim)) + round4k(gk_bytes(sim));
}

int tflbm_adj_seed(tflbm_sim *sim, void *d_adj, const double *d_grad_h, tflbm_stream_t stream) {
  if (!sim || !d_adj || !d_grad_h || ((uintptr_t)d_adj & 255) != 0) return TFLBM_EINVAL;
  if (!sim->initialised) return TFLBM_ESTATE;
  if (sim->kfield == kGammaKappa) {
    sim->last_error = "the reverse pass does not take a position-dependent surface tension (params.gamma_field)";
    return TFLBM_EINVAL;
  }
  sim->adj_cur = 1;  // seed writes the "dst" of a cur=1 state, i.e. the first buffer
  AdjArgs B = make_adj_args(sim, d_adj);
  const int rc = hip_status(sim, launch_adj_seed(sim->p.prec, B, d_grad_h, sim->w1, (hipStream_t)stream));
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
  const int rc = hip_status(sim, launch_adj_step(sim->p.prec, B, sim->kfield == kKappa, 1, sim->w1, (hipStream_t)stream));
  if (rc) return rc;
  sim->adj_cur ^= 1;
  return TFLBM_OK;
}

int tflbm_adj_steps(tflbm_sim *sim, void *d_adj, const void *d_capture, int64_t nsteps, tflbm_stream_t stream) {
  if (!sim || !d_adj || nsteps < 0 || (nsteps > 0 && !d_capture)) return TFLBM_EINVAL;
  if (!sim->adj_seeded) return TFLBM_ESTATE;
  const size_t cb = tflbm_capture_bytes(sim);
  const char *cap = (const char *)d_capture;
  int64_t t = nsteps - 1;
  while (t >= 0) {
    const bool fuse = sim->adj_fuse == 2 || (sim->adj_fuse == 0 && sim->adj_fuse_fits);
    const int ns = (t >= 1 && fuse) ? 2 : 1;
    AdjArgs B = make_adj_args(sim, d_adj, ns);
    B.cap = cap + (size_t)t * cb;
    B.cap2 = ns == 2 ? cap + (size_t)(t - 1) * cb : nullptr;
    const int rc = hip_status(sim, launch_adj_step(sim->p.prec, B, sim->kfield == kKappa, ns, sim->w1, (hipStream_t)stream));
    if (rc) return rc;
    sim->adj_cur ^= 1;
    t -= ns;
  }
  return TFLBM_OK;
}

int tflbm_adj_finish(tflbm_sim *sim, const void *d_adj, const double *d_h0, const double *d_theta,
                     double *d_grad_h0, double *d_grad_theta, tflbm_stream_t stream) {
  if (!sim || !d_adj) return TFLBM_EINVAL;
  if (d_grad_h0 && !d_h0) return TFLBM_EINVAL;
  if (!sim->adj_seeded) return TFLBM_ESTATE;
  AdjArgs B = make_adj_args(sim, (void *)d_adj);
  return hip_status(sim, launch_adj_finish(sim->p.prec, B, d_h0, d_theta, sim->p.theta0, sim->kconst, d_grad_h0,
                                           d_grad_theta, sim->w1, (hipStream_t)stream));
}

}  // extern "C"
