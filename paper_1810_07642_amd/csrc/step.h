// The fused step kernel and its launch templates (internal to the library),
// instantiated per storage form and collision stage in step_form.hip, which
// the build compiles once for each pair, so that they compile in parallel.
//
// Forward step of the thin-film lattice Boltzmann method (arXiv:1810.07642,
// Sec. II).
//
// Layout (HBM): population records of B consecutive columns of a row, all
// nine populations of the record contiguous, two buffers ping-pong (see
// device.h).  Population l of site (x, y) is stored in row y at column
// x - c_lx: streaming in y is a push (a row writes into rows y - 1, y, y + 1)
// and streaming in x is a pull (each lane reads its left or right
// neighbour's value), so every lane stores exactly its own columns and every
// store of a wavefront covers whole 128-byte lines of a record.
//
// Step kernel: one wavefront owns one record column (B output columns) plus a
// halo of (64 V - B)/2 columns per side (9 FP64, 10 FP32, 6 FP16S: three per
// fused step), and a chunk of H rows, and marches down the rows.  Per row it
// reads the nine segments of the row's records (coalesced, prefetched one to
// three rows ahead), assembles the deviations of its own columns (x shift
// through a cross-lane move), forms dh; one row later the film pressure of
// the previous row (Laplacian and disjoining term), kept as its x difference
// and x-smoothed value; one more row later the isotropic pressure gradient,
// forces, equilibrium and collision of the row two above, whose populations
// (or, with omega = 1, only their j) wait in LDS, and stores them.  Stencil
// neighbours in x come from adjacent lanes; no barriers.  With NS fused steps
// (two, or three with omega = 1) further such stages consume the previous
// one's output rows in registers, so every record crosses HBM once per NS
// steps; the halo columns and the 2 (2 + 3 (NS - 1)) halo rows of a chunk are
// re-read (partly from L2).
#pragma once

#include <type_traits>

#include "device.h"
#include "launch.h"

namespace tflbm {

// Loads the stored deviations d_l = f_l - E_l(href) of population l at the
// lane's columns of one row (resource `row`); oe/o16 are the lane's byte
// offsets in a segment of the working type (FP32 or FP64) and in an FP16
// segment; the segment offset is a compile-time immediate.  FP16S moving
// populations stay in their stored form, the FP16 words of the lane's two
// columns packed in out[0] (column 0 in the low half; out[1] unused), and are
// decoded only where the row is consumed (unpack16): a conversion here would
// make the prefetch of a row wait for its own loads.
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
      static_assert(V == 2, "FP16S packs the two columns of a lane in one word");
      if (vec) {
        out[0] = __uint_as_float(__builtin_bit_cast(unsigned int, ld_f16x2(row, o16[0] + seg)));
      } else {
        out[0] = __uint_as_float(__builtin_bit_cast(unsigned int, __halves2half2(ld_f16(row, o16[0] + seg), ld_f16(row, o16[1] + seg))));
      }
      out[1] = 0.0f;
    }
  }
}

// Per-lane geometry of a marching strip.
template <int P> struct Lane {
  static constexpr int V = Form<P>::V;
  int col[V];         // lattice column of each of the lane's V columns
  int oe[V], o16[V];  // byte offset in a row of records: working-type and FP16 segments
  int oc[V];          // byte offset in a row of capture records
  bool out[V];        // the column is an output of this strip
  bool vec;           // the column pair lies in one record, 8-byte aligned
  bool vecp;          // the column pair is contiguous and aligned in a plane array
  bool allvec;        // wave-uniform: vec on every lane
  bool allvecp;       // wave-uniform: vecp on every lane
  bool pair;          // all V columns are outputs and vec holds
  bool fast_store;    // wave-uniform: every lane has all or none of its columns as outputs, with vec
};

// Loads the stored deviations of all nine populations of one row.  Strips
// whose lanes all hold aligned column pairs (every strip of a lattice whose
// width is a multiple of the record size, and all interior strips otherwise)
// take the wave-uniform vector path with no per-lane branches.
template <int P>
__device__ __forceinline__ void load_row(rsrc_t row, const Lane<P> &L, typename Form<P>::T (&out)[9][Form<P>::V],
                                         const StepArgs &A) {
  if (L.allvec) {
#pragma unroll
    for (int l = 0; l < 9; ++l) load_raw<P>(row, l, L.oe, L.o16, true, out[l], A);
  } else {
#pragma unroll
    for (int l = 0; l < 9; ++l) load_raw<P>(row, l, L.oe, L.o16, L.vec, out[l], A);
  }
}

// FP32 rows in flight are held as one 64-bit word per population (the
// lane's two columns, column 0 in the low half), the shape of the 8-byte
// load: a 64-bit value keeps its aligned register pair up to the point the
// row is consumed, so the load writes those registers directly and nothing
// waits for it before then (held as two floats, the x shift of the consumer
// leads the register allocator to swap the pair with moves that wait).
__device__ __forceinline__ void load_row(rsrc_t row, const Lane<kF32> &L, unsigned long long (&out)[9]) {
  if (L.allvec) {
#pragma unroll
    for (int l = 0; l < 9; ++l)
      out[l] = __builtin_bit_cast(unsigned long long,
                                  __builtin_amdgcn_raw_buffer_load_b64(row, L.oe[0] + seg_offset<kF32>(l), 0, kLoadPolicy));
  } else {
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const int seg = seg_offset<kF32>(l);
      if (L.vec) {
        out[l] = __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(row, L.oe[0] + seg, 0, kLoadPolicy));
      } else {
        const u32x2 w = {__builtin_amdgcn_raw_buffer_load_b32(row, L.oe[0] + seg, 0, kLoadPolicy),
                         __builtin_amdgcn_raw_buffer_load_b32(row, L.oe[1] + seg, 0, kLoadPolicy)};
        out[l] = __builtin_bit_cast(unsigned long long, w);
      }
    }
  }
}

// FP32 rows of a strip whose lanes all hold aligned column pairs: nine 64-bit
// loads and no per-lane branch.
__device__ __forceinline__ void load_row_vec(rsrc_t row, const Lane<kF32> &L, unsigned long long (&out)[9]) {
#pragma unroll
  for (int l = 0; l < 9; ++l)
    out[l] = __builtin_bit_cast(unsigned long long,
                                __builtin_amdgcn_raw_buffer_load_b64(row, L.oe[0] + seg_offset<kF32>(l), 0, kLoadPolicy));
}

// FP16S rows of a strip whose lanes all hold aligned column pairs: the rest
// slot as one 64-bit load, each moving population as one 32-bit word of two
// FP16 values (as load_raw's vector path), no per-lane branch.
__device__ __forceinline__ void load_row_vec16(rsrc_t row, const Lane<kF16S> &L, float (&out)[9][2]) {
  const float2 v = ld_f32x2(row, L.oe[0] + seg_offset<kF16S>(0));
  out[0][0] = v.x;
  out[0][1] = v.y;
#pragma unroll
  for (int l = 1; l < 9; ++l) {
    out[l][0] = __uint_as_float(__builtin_bit_cast(unsigned int, ld_f16x2(row, L.o16[0] + seg_offset<kF16S>(l))));
    out[l][1] = 0.0f;
  }
}

// Per-site field of the film pressure (field kind KF):
//   kNoField: none (uniform kappa0 and gamma);
//   kKappa: kappa [ny][ldx] in T;
//   kGammaKappa: the pair (a, b) = (-gamma/6, -gamma kappa) per site, [ny][ldx][2]
//   in T, for a position-dependent surface tension (p = a 6 lap h + b phi(h)).
// The values of a lane's columns of one row travel with the rows: FP32 kappa
// as one 64-bit word (two columns, column 0 in the low half), FP32 pairs as
// one 128-bit word (a0 b0 a1 b1), FP64 kappa as one double, FP64 pairs as one
// 128-bit word (a, b); kappa_cols splits them into columns.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));
template <int P, int KF>
using KapBuf = std::conditional_t<KF == kGammaKappa, u32x4v,
                                  std::conditional_t<Form<P>::V == 2, unsigned long long, double>>;
template <int P, int KF> __device__ __forceinline__ void load_kappa(rsrc_t krow, const Lane<P> &L, KapBuf<P, KF> &out) {
  if constexpr (KF == kGammaKappa) {
    if constexpr (Form<P>::V == 2) {
      if (L.allvecp || L.vecp) {
        out = __builtin_bit_cast(u32x4v, __builtin_amdgcn_raw_buffer_load_b128(krow, L.col[0] * 8, 0, kLoadPolicy));
      } else {
        const u32x2 w0 = __builtin_amdgcn_raw_buffer_load_b64(krow, L.col[0] * 8, 0, kLoadPolicy);
        const u32x2 w1 = __builtin_amdgcn_raw_buffer_load_b64(krow, L.col[1] * 8, 0, kLoadPolicy);
        out = u32x4v{w0.x, w0.y, w1.x, w1.y};
      }
    } else {
      out = __builtin_bit_cast(u32x4v, __builtin_amdgcn_raw_buffer_load_b128(krow, L.col[0] * 16, 0, kLoadPolicy));
    }
  } else if constexpr (Form<P>::V == 2) {
    if (L.allvecp || L.vecp) {
      out = __builtin_bit_cast(unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(krow, L.col[0] * 4, 0, kLoadPolicy));
    } else {
      const u32x2 w = {__builtin_amdgcn_raw_buffer_load_b32(krow, L.col[0] * 4, 0, kLoadPolicy),
                       __builtin_amdgcn_raw_buffer_load_b32(krow, L.col[1] * 4, 0, kLoadPolicy)};
      out = __builtin_bit_cast(unsigned long long, w);
    }
  } else {
    out = ld_f64(krow, L.col[0] * 8);
  }
}
// Splits a row's field values into the kappa slot k (kappa, or b = -gamma
// kappa) and, for kGammaKappa, a = -gamma/6.
template <int P, int KF>
__device__ __forceinline__ void kappa_cols(const KapBuf<P, KF> &k, typename Form<P>::T (&out)[Form<P>::V],
                                           typename Form<P>::T (&aco)[Form<P>::V]) {
  if constexpr (KF == kGammaKappa) {
    if constexpr (Form<P>::V == 2) {
      aco[0] = __uint_as_float(k.x);
      out[0] = __uint_as_float(k.y);
      aco[1] = __uint_as_float(k.z);
      out[1] = __uint_as_float(k.w);
    } else {
      aco[0] = __longlong_as_double(((long long)k.y << 32) | k.x);
      out[0] = __longlong_as_double(((long long)k.w << 32) | k.z);
    }
  } else if constexpr (Form<P>::V == 2) {
    const u32x2 w = __builtin_bit_cast(u32x2, k);
    out[0] = __uint_as_float(w.x);
    out[1] = __uint_as_float(w.y);
  } else {
    out[0] = k;
  }
}

// Step constants in the working type.
template <typename T> struct Coef {
  T omega, om1, nu, hstar, href, g, ax, ay, kap0, cA, cD, three_delta2, six_delta, mgam, mgam6;
  int n_exp, m_exp;
  __device__ explicit Coef(const StepArgs &A) {
    omega = (T)A.omega;
    om1 = (T)(1.0 - A.omega);
    nu = (T)A.nu;
    hstar = (T)A.hstar;
    href = (T)A.href;
    g = (T)A.g;
    ax = (T)A.ax;
    ay = (T)A.ay;
    kap0 = (T)A.kappa0;
    cA = (T)(3.0 * kW[1]);  // gradient stencil weight on the axes (1/3)
    cD = (T)(3.0 * kW[2]);  // and on the diagonals (1/12)
    three_delta2 = (T)(3.0 * A.delta * A.delta);
    six_delta = (T)(6.0 * A.delta);
    mgam = (T)(-A.gamma);
    mgam6 = (T)(-A.gamma / 6.0);
    n_exp = A.n_exp;
    m_exp = A.m_exp;
  }
};

// Values of population l at the lane's own columns, from a row of values held
// at columns x - c_lx (stored records, or post-collision values before their
// x streaming): the x shift is a move from the neighbouring lane.
template <typename T, int V>
__device__ __forceinline__ void shift_x(int l, const T *in, T *out) {
  if (kCx[l] == 0) {
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = in[v];
  } else if (kCx[l] > 0) {
    out[0] = from_left(in[V - 1]);
#pragma unroll
    for (int v = 1; v < V; ++v) out[v] = in[v - 1];
  } else {
#pragma unroll
    for (int v = 0; v < V - 1; ++v) out[v] = in[v + 1];
    out[V - 1] = from_right(in[0]);
  }
}

// One time step applied row by row to a marching strip.  ingest(k, ...)
// takes the pre-collision deviations d_l = f_l - E_l(href) of the stage's
// k-th row r and forms dh = h - href = sum d; finish(k, ...) forms the film
// pressure of row r-1 and, for k >= 4, the post-collision deviations of row
// r-2 (eqs. "LBE", "equilibria", "force", "pfilm", "disjoiningP",
// "forcefric", "alphafric", "derivative", "n_laplace").  The populations of
// rows r-1 and r-2 wait in two LDS slots.  The shift by E_l(href) is constant,
// has zero momentum and is a fixed point of the collision at rest, so the
// step on d is the step on f; only small changes of a film near href keep
// more significant digits.
// W1 (omega = 1, tau = 1): BGK replaces the populations by the equilibrium,
// so the emitted row needs only its moments: j is formed at ingest and waits
// two rows in an LDS slot of two values per column (instead of nine), and
// no populations are kept.  The values are those of the general stage bit
// for bit: with 1 - omega = 0 its term (1 - omega) d adds an exact zero.
template <int P, int KF, bool W1 = false> struct Stage {
  using T = typename Form<P>::T;
  static constexpr int V = Form<P>::V;
  T h0[V + 2], h1[V + 2], h2[V + 2];  // dh of rows r, r-1, r-2 with the left/right neighbours
  // per row of p: x difference p(x+1) - p(x-1) and the x-smoothed value
  // cA p(x) + cD (p(x-1) + p(x+1)), of rows r-1, r-2, r-3
  T dx1[V], dx2[V], dx3[V];
  T sm1[V], sm2[V], sm3[V];
  T kn[V], kr[V];                     // kappa (or -gamma kappa) of rows r and r-1
  T an[V], ar[V];                     // -gamma/6 of rows r and r-1 (kGammaKappa)
  T jx2[V], jy2[V];                   // W1: j of row r-2, from ingest to finish
  T (*hist)[9][64 * V];               // general: populations of rows r-1, r-2 [slot][l][column]
  T (*jhist)[2][64 * V];              // W1: j of rows r-1, r-2 [slot][x or y][column]

  // kap, aco: the field values of row r (loaded with the row, load_kappa;
  // unused without a field)
  __device__ __forceinline__ void ingest(int k, const T (&f)[9][V], const T (&kap)[V], const T (&aco)[V],
                                         T (&f2)[9][V], int lane) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T hs = f[0][v];
#pragma unroll
      for (int l = 1; l < 9; ++l) hs += f[l][v];
      h0[1 + v] = hs;
    }
    h0[0] = from_left(h0[V]);
    h0[V + 1] = from_right(h0[1]);
    // kappa of row r, used by the pressure of row r at the next row
#pragma unroll
    for (int v = 0; v < V; ++v) {
      kr[v] = kn[v];
      if constexpr (KF != kNoField) kn[v] = kap[v];
      if constexpr (KF == kGammaKappa) {
        ar[v] = an[v];
        an[v] = aco[v];
      }
    }
    if constexpr (W1) {
      // j = sum_l c_l d_l through the differences of opposite populations;
      // row r-2's leaves the slot that row r's takes over
      const int slot = k & 1;
      if (k >= 4) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          jx2[v] = jhist[slot][0][V * lane + v];
          jy2[v] = jhist[slot][1][V * lane + v];
        }
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T d15 = f[1][v] - f[5][v], d37 = f[3][v] - f[7][v];
        const T d26 = f[2][v] - f[6][v], d84 = f[8][v] - f[4][v];
        jhist[slot][0][V * lane + v] = (d15 + d26) + d84;
        jhist[slot][1][V * lane + v] = (d37 + d26) - d84;
      }
    } else {
      // row r-2 leaves the LDS slot that row r takes over
      const int slot = k & 1;
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
    }
  }

  __device__ __forceinline__ bool finish(int k, const T (&f2)[9][V], T (&post)[9][V], T (&hv)[V], T (&jxv)[V],
                                         T (&jyv)[V], const Coef<T> &C, const Lane<P> &L, int &bad) {
    if (k >= 2) {
      // film pressure of row r-1: p = -gamma (lap h + kappa phi(h))
      T pc[V + 2];
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
        const T hc = C.href + h1[v + 1];
        // 6 lap h = 6 lap dh = 4 sum_axes + sum_diagonals - 20 dh
        const T lap6 = madd(T(-20), h1[v + 1], madd(T(4), odd, even));
        const T phi = disjoining(C.hstar * recip(hc), C.n_exp, C.m_exp);
        if constexpr (KF == kGammaKappa) {
          // per-site (-gamma/6, -gamma kappa), rounded at init as the scalar
          // path rounds (-gamma/6) and (-gamma) kappa
          pc[v + 1] = madd(ar[v], lap6, kr[v] * phi);
        } else {
          const T kap = KF == kKappa ? kr[v] : C.kap0;
          pc[v + 1] = madd(C.mgam6, lap6, C.mgam * kap * phi);
        }
      }
      pc[0] = from_left(pc[V]);
      pc[V + 1] = from_right(pc[1]);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        dx1[v] = pc[v + 2] - pc[v];
        sm1[v] = madd(C.cA, pc[v + 1], C.cD * (pc[v] + pc[v + 2]));
      }
    }
    const bool emit = k >= 4;
    if (emit) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // isotropic gradient of p: axis weight 1/3, diagonal 1/12
        const T gx = madd(C.cA, dx2[v], C.cD * (dx1[v] + dx3[v]));
        const T gy = sm1[v] - sm3[v];

        const T dh = h2[1 + v];
        const T h = C.href + dh;
        T jx, jy;
        if constexpr (W1) {
          jx = jx2[v];
          jy = jy2[v];
        } else {
          // j = sum_l c_l d_l through the differences of opposite populations
          const T d15 = f2[1][v] - f2[5][v], d37 = f2[3][v] - f2[7][v];
          const T d26 = f2[2][v] - f2[6][v], d84 = f2[8][v] - f2[4][v];
          jx = (d15 + d26) + d84;
          jy = (d37 + d26) - d84;
        }
        const T inv_h = recip(h);
        const T ux = jx * inv_h, uy = jy * inv_h;

        // F = h (a - grad p) - nu alpha(h) u, alpha = 6 h / (2 h^2 + 6 delta h + 3 delta^2)
        const T alpha = T(6) * h * recip(madd(T(2) * h, h, madd(C.six_delta, h, C.three_delta2)));
        const T fric = C.nu * alpha;
        const T Fx = madd(h, C.ax - gx, -fric * ux);
        const T Fy = madd(h, C.ay - gy, -fric * uy);

        // equilibrium (lattice speed 1 in the printed denominators) minus the
        // stored shift E_l(href, 0), with q = g (h^2 - href^2) = g dh (h + href):
        //   rest: dh - 5 q/6 - 2 h u^2/3
        //   axes: q/6 + h ((c.u)/3 + (c.u)^2/2 - u^2/6)
        //   diagonals: q/24 + h ((c.u)/12 + (c.u)^2/8 - u^2/24)
        // BGK with forcing: d + omega (deq - d) + 3 w_l c_l.F.  Opposite
        // populations l, -l share the even part in c and differ in the sign of
        // the odd part: post = (1 - omega) d + E +- O with
        //   E = omega h ((c.u)^2 w2 - u^2 w0) + omega q w0,
        //   O = w1 (omega h c.u + c.F),  (w0, w1, w2) = (1/6, 1/3, 1/2) on the
        //   axes and (1/24, 1/12, 1/8) on the diagonals.
        const T usq = madd(ux, ux, uy * uy);
        const T hom = h * C.omega;
        const T G = C.omega * (C.g * dh * (h + C.href));  // omega q
        const T e0 = madd(hom, usq * T(-2.0 / 3.0), madd(G, T(-5.0 / 6.0), C.omega * dh));
        if constexpr (W1) post[0][v] = e0;
        else post[0][v] = madd(C.om1, f2[0][v], e0);
        const T evA = madd(hom, usq * T(-1.0 / 6.0), G * T(1.0 / 6.0));    // E without (c.u)^2, axes
        const T evD = madd(hom, usq * T(-1.0 / 24.0), G * T(1.0 / 24.0));  // and diagonals
        auto opposite = [&](int lp, int lm, T cu, T cF, T ev, T w1, T w2) {
          const T hc = hom * cu;
          const T E = madd(hc, cu * w2, ev);
          const T O = hc + cF;
          if constexpr (W1) {
            post[lp][v] = madd(O, w1, E);
            post[lm][v] = madd(-O, w1, E);
          } else {
            post[lp][v] = madd(O, w1, madd(C.om1, f2[lp][v], E));
            post[lm][v] = madd(-O, w1, madd(C.om1, f2[lm][v], E));
          }
        };
        opposite(1, 5, ux, Fx, evA, T(1.0 / 3.0), T(0.5));
        opposite(3, 7, uy, Fy, evA, T(1.0 / 3.0), T(0.5));
        opposite(2, 6, ux + uy, Fx + Fy, evD, T(1.0 / 12.0), T(0.125));
        opposite(4, 8, uy - ux, Fy - Fx, evD, T(1.0 / 12.0), T(0.125));
        hv[v] = dh;
        jxv[v] = jx;
        jyv[v] = jy;
        if (L.out[v] && !(h > T(0) && h < T(INFINITY))) bad = 1;
      }
    }
#pragma unroll
    for (int v = 0; v < V + 2; ++v) {
      h2[v] = h1[v];
      h1[v] = h0[v];
    }

#pragma unroll
    for (int v = 0; v < V; ++v) {
      dx3[v] = dx2[v];
      dx2[v] = dx1[v];
      sm3[v] = sm2[v];
      sm2[v] = sm1[v];
    }
    return emit;
  }
};

// Two values scaled by 2^s and rounded to FP16 (round to nearest even), packed
// in one word, the first in the low half: the stored form of a lane's two
// columns.  The scale is a power of two, so the product is exact and the one
// rounding is the conversion's (the same bits as __float2half_rn of the
// product, which the round trip of the fused pass uses).
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned int enc16x2(float a, float b, float qscale) {
  f16x2_t w;
  w.x = (_Float16)(a * qscale);
  w.y = (_Float16)(b * qscale);
  return __builtin_bit_cast(unsigned int, w);
}

// A buffer offset past every row (kDropBytes): an access there is dropped by
// the buffer range check and touches no memory.
constexpr int kStoreDrop = kDropBytes;

// Uniform stores.  The counter a wavefront waits on for its loads also counts
// its stores and retires both in issue order, and the compiler sizes each
// wait for the path through the loop with the fewest memory instructions
// after the load.  A row iteration whose stores are skipped on some path (a
// lane mask that may be empty, a stage that has not started emitting) makes
// the wait for the next prefetched row drain the stores just issued, so every
// row pays the latency of its own stores.  With UNI, store_row issues the
// same stores on every path (lanes that store nothing aim at kStoreDrop), the
// iterations before the first stored row issue as many dropped stores
// (drop_row_stores), and the row loop tells the compiler which iterations
// store: the wait for a row then leaves the previous row's stores in flight.
// Measured (FP64 MLUPS, bitwise the same results): three omega = 1 steps per
// pass at 4096^2 72.4k -> 77.9k, at 2048^2 63.6k -> 69.8k; the general stages
// (two steps) at 4096^2 54.5k -> 57.9k.  Left out where it lost: the one- and
// two-step omega = 1 kernels of small lattices, whose tiles are bound by their
// chain of rows (256^2 10.3k -> 9.1k), and FP32 and FP16S outside the aligned
// specialisation of their main kernels (step_kernel's row loop; with the
// per-lane load branches of the general loop FP32 ran 2 % and FP16S 5 %
// slower, in it 2 % and 5 % faster); the capture and surface tension kernels
// would spill.
template <int P> __device__ __forceinline__ void drop_row_stores(const StepArgs &A) {
  // byte stores at distinct offsets: a store of this width occurs nowhere
  // else, so the compiler neither merges these with a row's stores nor drops
  // them as duplicates
  const rsrc_t none = make_rsrc(A.dst, 0);
#pragma unroll
  for (int i = 0; i < 12; ++i) __builtin_amdgcn_raw_buffer_store_b8((unsigned char)0, none, kStoreDrop + 4 * i, 0, kStorePolicy);
}

// Stores the post-collision deviations of row y (values at the lane's own
// columns, hv = dh of the row) into stored column x of rows y + c_ly; UNI:
// uniform stores (above), FP64 only.
template <int P, bool G0 = false, bool UNI = false>
__device__ __forceinline__ void store_row(const StepArgs &A, int y, const typename Form<P>::T (&post)[9][Form<P>::V],
                                          const typename Form<P>::T (&hv)[Form<P>::V], const Lane<P> &L, int x0,
                                          int xend, int lane) {
  constexpr int V = Form<P>::V;
  constexpr int B = Form<P>::B;
  constexpr int RB = Form<P>::RB;
  const int ny = A.ny;
  const size_t rowB = (size_t)A.nblk * RB;
  const int yN = (y + 1 == ny) ? 0 : y + 1;
  const int yS = (y == 0) ? ny - 1 : y - 1;
  const rsrc_t rowD[3] = {make_rsrc(A.dst + yS * rowB, (uint32_t)rowB), make_rsrc(A.dst + y * rowB, (uint32_t)rowB),
                          make_rsrc(A.dst + yN * rowB, (uint32_t)rowB)};  // indexed by c_ly + 1
  const bool pair = L.pair;
  if constexpr (UNI && P != kF16S) {
    // nine stores and three padding stores on every path (FP32: only where
    // every lane stores both of its columns or none, fast_store)
    if constexpr (P == kF64) {
      const int oe = L.out[0] ? L.oe[0] : kStoreDrop;  // one column per lane: pair == out[0]
#pragma unroll
      for (int l = 0; l < 9; ++l) st_f64(rowD[kCy[l] + 1], oe + seg_offset<P>(l), post[l][0]);
    } else {
      const int oe = pair ? L.oe[0] : kStoreDrop;
#pragma unroll
      for (int l = 0; l < 9; ++l) st_f32x2(rowD[kCy[l] + 1], oe + seg_offset<P>(l), post[l][0], post[l][1]);
    }
    const bool full = xend - x0 == B;
    const int rec = (x0 / B) * RB;
#pragma unroll
    for (int g = 0; g < 3; ++g)
      st_f32(rowD[g == 0 ? 1 : (g == 1 ? 2 : 0)],
             full && 4 * lane < pad_bytes<P>(g) ? rec + pad_offset<P>(g) + 4 * lane : kStoreDrop, 0.f);
    return;
  }
  if constexpr (P == kF16S) {
    // the site's height deviation s, and each moving population as its FP16
    // difference from the rest equilibrium e_l(s) of this (its source) site,
    // the lane's two columns packed in one word (column 0 in the low half)
    static_assert(V == 2, "FP16S packs the two columns of a lane in one word");
    float rest[V];
    unsigned int qw[9];
    const float g16 = (float)A.g, h2 = 2.0f * (float)A.href;
#pragma unroll
    for (int v = 0; v < V; ++v) rest[v] = hv[v];
    if constexpr (G0) {  // g = 0: the rest equilibrium has no moving part
#pragma unroll
      for (int l = 1; l < 9; ++l) qw[l] = enc16x2(post[l][0], post[l][1], A.qscale);
    } else {
      const Rest16 e0 = rest16(hv[0], g16, h2), e1 = rest16(hv[1], g16, h2);
#pragma unroll
      for (int l = 1; l < 9; ++l)
        qw[l] = enc16x2(post[l][0] - rest16_l(e0, l), post[l][1] - rest16_l(e1, l), A.qscale);
    }
    if constexpr (UNI) {
      const int o16 = pair ? L.o16[0] : kStoreDrop, oe = pair ? L.oe[0] : kStoreDrop;
#pragma unroll
      for (int l = 1; l < 9; ++l)
        __builtin_amdgcn_raw_buffer_store_b32(qw[l], rowD[kCy[l] + 1], o16 + seg_offset<P>(l), 0, kStorePolicy);
      st_f32x2(rowD[1], oe, rest[0], rest[1]);
      const bool full = xend - x0 == B;
      const int rec = (x0 / B) * RB;
#pragma unroll
      for (int g = 0; g < 3; ++g)
        st_f32(rowD[g == 0 ? 1 : (g == 1 ? 2 : 0)],
               full && 4 * lane < pad_bytes<P>(g) ? rec + pad_offset<P>(g) + 4 * lane : kStoreDrop, 0.f);
      return;
    } else if (L.fast_store) {
      if (pair) {
#pragma unroll
        for (int l = 1; l < 9; ++l)
          __builtin_amdgcn_raw_buffer_store_b32(qw[l], rowD[kCy[l] + 1], L.o16[0] + seg_offset<P>(l), 0, kStorePolicy);
        st_f32x2(rowD[1], L.oe[0], rest[0], rest[1]);
      }
    } else {
#pragma unroll
      for (int l = 1; l < 9; ++l) {
        const rsrc_t rd = rowD[kCy[l] + 1];
        const int seg = seg_offset<P>(l);
        if (pair) {
          __builtin_amdgcn_raw_buffer_store_b32(qw[l], rd, L.o16[0] + seg, 0, kStorePolicy);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (L.out[v]) st_f16(rd, L.o16[v] + seg, __ushort_as_half((unsigned short)(v ? qw[l] >> 16 : qw[l] & 0xffffu)));
        }
      }
      if (pair) {
        st_f32x2(rowD[1], L.oe[0], rest[0], rest[1]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (L.out[v]) st_f32(rowD[1], L.oe[v], rest[v]);
      }
    }
  } else if (L.fast_store) {
    // every lane stores all of its columns or none: one masked region
    if (pair) {
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        const rsrc_t rd = rowD[kCy[l] + 1];
        if constexpr (P == kF64) st_f64(rd, L.oe[0] + seg_offset<P>(l), post[l][0]);
        else st_f32x2(rd, L.oe[0] + seg_offset<P>(l), post[l][0], post[l][1]);
      }
    }
  } else {
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      const rsrc_t rd = rowD[kCy[l] + 1];
      const int seg = seg_offset<P>(l);
      if constexpr (P == kF64) {
        if (L.out[0]) st_f64(rd, L.oe[0] + seg, post[l][0]);
      } else {
        if (pair) {
          st_f32x2(rd, L.oe[0] + seg, post[l][0], post[l][1]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (L.out[v]) st_f32(rd, L.oe[v] + seg, post[l][v]);
        }
      }
    }
  }
  // zero the padding after each c_ly group of a full record so that its
  // lines are written whole
  if (xend - x0 == B) {
    const int rec = (x0 / B) * RB;
#pragma unroll
    for (int g = 0; g < 3; ++g)
      if (4 * lane < pad_bytes<P>(g)) st_f32(rowD[g == 0 ? 1 : (g == 1 ? 2 : 0)], rec + pad_offset<P>(g) + 4 * lane, 0.f);
  }
}

// FP16S storage round trip of one row of post-collision deviations (what a
// store followed by a load would give): moving deviations rounded to FP16 as
// differences from the rest equilibrium of the writing site, rest deviation
// implied by its height deviation hv (rest16_d0).
template <int V, bool G0>
__device__ __forceinline__ void fp16s_roundtrip(float (&post)[9][V], const float (&hv)[V], const StepArgs &A) {
  const float g16 = (float)A.g, h2 = 2.0f * (float)A.href;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    float d[9];
    d[0] = 0.0f;
    if constexpr (G0) {
#pragma unroll
      for (int l = 1; l < 9; ++l) d[l] = dec16(__float2half_rn(post[l][v] * A.qscale), A.qinv);
    } else {
      const Rest16 e = rest16(hv[v], g16, h2);
#pragma unroll
      for (int l = 1; l < 9; ++l) {
        const float el = rest16_l(e, l);
        d[l] = el + dec16(__float2half_rn((post[l][v] - el) * A.qscale), A.qinv);
      }
    }
#pragma unroll
    for (int l = 1; l < 9; ++l) post[l][v] = d[l];
    post[0][v] = rest16_d0(hv[v], d);
  }
}

// Scaled-back FP16 difference of column v from a word of two packed FP16
// values (load_raw).
__device__ __forceinline__ float unpack16(float w, int v, float qinv) {
  const unsigned int u = __float_as_uint(w);
  return dec16(__ushort_as_half((unsigned short)(v ? (u >> 16) : (u & 0xffffu))), qinv);
}

// FP16S decoding of stored row r (slot 0 the site's s, slots l >= 1 the
// packed FP16 differences) into deviations, per stored column: moving
// populations add the rest equilibrium of their source row (r for c_ly = 0,
// r - 1 for +1, r + 1 for -1); the rest deviation of row r's sites is implied
// by their s and the moving populations they emitted, which sit in rows r
// (c_ly = 0), r + 1 (+1) and r - 1 (-1, kept from the previous row as cq
// together with its s, cs).  The c_ly = +1 values of row r were decoded for
// the previous row and come in cn.  On return cs, cq and cn hold the values
// the next row needs.
template <int V, bool G0>
__device__ __forceinline__ void fp16s_decode(const float (&cur)[9][V], const float (&nxt)[9][V], float (&cs)[V],
                                             float (&cq)[3][V], float (&cn)[3][V], const StepArgs &A,
                                             float (&d)[9][V]) {
  const float g16 = (float)A.g, h2 = 2.0f * (float)A.href;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    float qc[9], qn[9], t[9];
#pragma unroll
    for (int l = 1; l < 9; ++l) {
      qc[l] = kCy[l] > 0 ? cn[l - 2][v] : unpack16(cur[l][0], v, A.qinv);
      qn[l] = kCy[l] > 0 ? unpack16(nxt[l][0], v, A.qinv) : 0.0f;
    }
    t[0] = 0.0f;
    if constexpr (G0) {  // g = 0: the values are the differences themselves
#pragma unroll
      for (int l = 1; l < 9; ++l) {
        d[l][v] = qc[l];
        t[l] = kCy[l] == 0 ? qc[l] : (kCy[l] > 0 ? qn[l] : cq[l >= 6 ? l - 6 : 0][v]);
      }
    } else {
      const Rest16 em = rest16(cs[v], g16, h2), e0 = rest16(cur[0][v], g16, h2), ep = rest16(nxt[0][v], g16, h2);
#pragma unroll
      for (int l = 1; l < 9; ++l) {
        const Rest16 &e = kCy[l] == 0 ? e0 : (kCy[l] > 0 ? em : ep);
        d[l][v] = rest16_l(e, l) + qc[l];
        const float qo = kCy[l] == 0 ? qc[l] : (kCy[l] > 0 ? qn[l] : cq[l >= 6 ? l - 6 : 0][v]);
        t[l] = rest16_l(e0, l) + qo;
      }
    }
    d[0][v] = rest16_d0(cur[0][v], t);
    cs[v] = cur[0][v];
    cq[0][v] = qc[6];
    cq[1][v] = qc[7];
    cq[2][v] = qc[8];
    cn[0][v] = qn[2];
    cn[1][v] = qn[3];
    cn[2][v] = qn[4];
  }
}

// Moments (h, jx, jy) of row q of the pre-collision state of one step, for
// the reverse sweep, into the capture records at `base` (cap_record_bytes).
// UNI (the aligned FP32 copy of the row loop, where every lane stores both of
// its columns or neither): the same four stores on every path, lanes without
// output and rows outside the tile (`valid` false: an empty range) dropped.
template <int P, bool UNI = false>
__device__ __forceinline__ void capture_row(const StepArgs &A, char *base, int q, const typename Form<P>::T (&hv)[Form<P>::V],
                                            const typename Form<P>::T (&jxv)[Form<P>::V],
                                            const typename Form<P>::T (&jyv)[Form<P>::V], const Lane<P> &L,
                                            typename Form<P>::T href, int x0, int xend, int lane, bool valid = true) {
  using T = typename Form<P>::T;
  constexpr int V = Form<P>::V, B = Form<P>::B, ES = sizeof(T);
  constexpr int CRB = cap_record_bytes<P>(), SEG = B * ES;
  const uint32_t rowb = (uint32_t)(A.nblk * CRB);
  const rsrc_t row = make_rsrc(base + (size_t)(valid ? q : 0) * rowb, valid ? rowb : 0u);
  if constexpr (UNI && V == 2) {
    const int oc = L.pair ? L.oc[0] : kStoreDrop;
    st_f32x2(row, oc, href + hv[0], href + hv[1]);
    st_f32x2(row, oc + SEG, jxv[0], jxv[1]);
    st_f32x2(row, oc + 2 * SEG, jyv[0], jyv[1]);
    st_f32(row, xend - x0 == B && 4 * lane < CRB - 3 * SEG ? (x0 / B) * CRB + 3 * SEG + 4 * lane : kStoreDrop, 0.f);
    return;
  }
  if constexpr (V == 2) {
    if (L.pair) {
      st_f32x2(row, L.oc[0], href + hv[0], href + hv[1]);
      st_f32x2(row, L.oc[0] + SEG, jxv[0], jxv[1]);
      st_f32x2(row, L.oc[0] + 2 * SEG, jyv[0], jyv[1]);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (L.out[v]) {
          st_t(row, L.oc[v], href + hv[v]);
          st_t(row, L.oc[v] + SEG, jxv[v]);
          st_t(row, L.oc[v] + 2 * SEG, jyv[v]);
        }
      }
    }
  } else {
    if (L.out[0]) {
      st_t(row, L.oc[0], href + hv[0]);
      st_t(row, L.oc[0] + SEG, jxv[0]);
      st_t(row, L.oc[0] + 2 * SEG, jyv[0]);
    }
  }
  // zero the padding of a full record so that its last line is written whole
  if (xend - x0 == B && 4 * lane < CRB - 3 * SEG) st_f32(row, (x0 / B) * CRB + 3 * SEG + 4 * lane, 0.f);
}

// Hands the post-collision rows of one stage to the next stage (the next time
// step) in registers: post-collision values waiting for the next step, already
// moved to their destination columns (the x part of streaming), are the
// c_ly = +1 populations of the last two emitted rows and the c_ly = 0
// populations of the last one.  feed() takes the row q just emitted and gives
// the complete pre-collision row q - 1 of the next step: c_ly = +1 populations
// from row q - 2, c_ly = 0 from row q - 1, c_ly = -1 from row q.
template <typename T, int V> struct Handoff {
  T pendP1[3][V], pendP2[3][V], pendZ[3][V];
  __device__ __forceinline__ void feed(const T (&post)[9][V], T (&g)[9][V]) {
    shift_x<T, V>(6, post[6], g[6]);
    shift_x<T, V>(7, post[7], g[7]);
    shift_x<T, V>(8, post[8], g[8]);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      g[2][v] = pendP2[0][v];
      g[3][v] = pendP2[1][v];
      g[4][v] = pendP2[2][v];
      g[0][v] = pendZ[0][v];
      g[1][v] = pendZ[1][v];
      g[5][v] = pendZ[2][v];
      pendP2[0][v] = pendP1[0][v];
      pendP2[1][v] = pendP1[1][v];
      pendP2[2][v] = pendP1[2][v];
    }
    shift_x<T, V>(2, post[2], pendP1[0]);
    shift_x<T, V>(3, post[3], pendP1[1]);
    shift_x<T, V>(4, post[4], pendP1[2]);
    shift_x<T, V>(0, post[0], pendZ[0]);
    shift_x<T, V>(1, post[1], pendZ[1]);
    shift_x<T, V>(5, post[5], pendZ[2]);
  }
};

// NS fused time steps per pass (1, 2 or 3).  Stage 0 consumes the stored rows;
// with NS >= 2 its post-collision rows are streamed in registers into stage 1
// (rows arrive one row late: row q of the next step needs the post-collision
// values of rows q-1, q, q+1), and with NS = 3 those of stage 1 into stage 2;
// the last stage's output is stored.  The strip's chunk reads 2 + 3 (NS - 1)
// halo rows above and below.  With CAP the moments of each step's
// pre-collision state on the tile's own rows go to the capture: step t at
// A.capture, step t + s s capture blocks later.
// G0 (FP16S only): the launch has g = 0, so the rest equilibrium of the
// FP16S shift has no moving part and its code is left out.
// W1: omega = 1, the stages keep no populations (Stage), only j of two rows
// in LDS, which lets three fused steps keep eight wavefronts per CU.
template <int P, int KF, bool CAP, int NS, bool G0 = false, bool W1 = false>
__global__ __launch_bounds__(64, 2) void step_kernel(StepArgs A) {
  using T = typename Form<P>::T;
  constexpr int V = Form<P>::V;
  constexpr int B = Form<P>::B;
  constexpr int RB = Form<P>::RB;
  constexpr int HX = (64 * V - B) / 2;  // halo columns per side (>= 3 NS)
  constexpr int ES = sizeof(T);
  static_assert(HX >= 3 * NS, "halo columns too narrow for the fused steps");
  // the stages' history of two rows: populations (general) or j (W1)
  __shared__ T hist[W1 ? 1 : NS][W1 ? 1 : 2][W1 ? 1 : 9][W1 ? 1 : 64 * V];
  __shared__ T jhist[W1 ? NS : 1][W1 ? 2 : 1][2][W1 ? 64 * V : 1];

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
  const int nx = A.nx, ny = A.ny;
  const size_t rowB = (size_t)A.nblk * RB;

  Lane<P> L;
  const int a = x0 - HX + V * lane;  // first (unwrapped) column of this lane
#pragma unroll
  for (int v = 0; v < V; ++v) {
    L.col[v] = wrap(a + v, nx);
    const int blk = L.col[v] / B;
    const int pos = L.col[v] - blk * B;
    L.oe[v] = blk * RB + pos * ES;
    L.oc[v] = blk * cap_record_bytes<P>() + pos * ES;
    L.o16[v] = blk * RB + pos * 2;
    L.out[v] = (a + v >= x0) && (a + v < xend);
  }
  L.vec = true;
  L.vecp = true;
  if constexpr (V == 2) {
    L.vec = (L.col[1] == L.col[0] + 1) && (L.col[0] / B == L.col[1] / B) && ((L.col[0] & 1) == 0);
    L.vecp = (L.col[1] == L.col[0] + 1) && ((L.col[0] & 1) == 0);
  }
  L.pair = L.out[0] && L.out[V - 1] && L.vec;
  L.allvec = __all(L.vec);
  L.allvecp = __all(L.vecp);
  L.fast_store = __all(L.pair || (!L.out[0] && !L.out[V - 1]));
  const Coef<T> C(A);

  Stage<P, KF, W1> S0, S1, S2;
  if constexpr (W1) {
    S0.jhist = jhist[0];
    if constexpr (NS >= 2) S1.jhist = jhist[1];
    if constexpr (NS >= 3) S2.jhist = jhist[2];
  } else {
    S0.hist = hist[0];
    if constexpr (NS >= 2) S1.hist = hist[1];
    if constexpr (NS >= 3) S2.hist = hist[2];
  }
  Handoff<T, V> H1, H2;  // stage 0 -> 1, stage 1 -> 2
  int bad = 0;
  const size_t capblk = (size_t)ny * A.nblk * cap_record_bytes<P>();

  constexpr int HALO = 2 + 3 * (NS - 1);
  const int K = (yend - y0) + 2 * HALO;
  // uniform stores (store_row) and KST, the first row iteration whose last
  // stage stores a row (each stage emits from its fifth row on, and stage s
  // starts six rows after stage s - 1)
  constexpr bool UNI64 = P == kF64 && !CAP && KF != kGammaKappa && (NS == 3 || !W1);
  constexpr int KST = 4 + 6 * (NS - 1);
  auto rsrc_src = [&](int row) { return make_rsrc(A.src + row * rowB, (uint32_t)rowB); };
  int ry = wrap(y0 - HALO, ny);                          // row r of stage 0
  // rows are loaded PF rows ahead of their use.  Measured at 4096^2 with two
  // fused steps (MLUPS, two rows ahead / three): FP16S 142.8k / 146.9k (its
  // decoding makes each row wait longer for its loads), FP32 113.9k / 113.3k,
  // FP64 57.9k / 58.0k.  The three-step kernels load one row ahead: two would
  // need more than 256 VGPRs.
  constexpr int PF = P == kF16S ? 3 : (NS == 3 ? 1 : 2);
  int rpre = (ry + PF) % ny;                             // row r + PF
  // FP16S decodes row r with rows r - 1 and r + 1 (fp16s_decode): the row
  // above the first is read for its s and q_6..q_8, and one row past the
  // last (KL = K + 1 rows are loaded after it)
  T cs[V], cq[3][V], cn[3][V];
  constexpr int KX = P == kF16S ? 1 : 0;
  const int KL = K + KX;
  if constexpr (P == kF16S) {
    T fp[9][V];
    load_row<P>(rsrc_src(ry == 0 ? ny - 1 : ry - 1), L, fp, A);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      cs[v] = fp[0][v];
      cq[0][v] = unpack16(fp[6][0], v, A.qinv);
      cq[1][v] = unpack16(fp[7][0], v, A.qinv);
      cq[2][v] = unpack16(fp[8][0], v, A.qinv);
    }
  }
  // kappa travels with the rows: ka and kb hold the kappa of the rows in fa
  // and fb, and stage 1, three rows behind stage 0, takes it from kq (the
  // kappa of stage 0's last three rows)
  const uint32_t kpitch = (uint32_t)(A.ldx * sizeof(T) * (KF == kGammaKappa ? 2 : 1));
  auto rsrc_kap = [&](int row) { return make_rsrc((const char *)A.kfield + (size_t)row * kpitch, kpitch); };
  KapBuf<P, KF> ka, kb, kc;
  // field values of stage 0's last rows, for the later stages (stage s runs
  // 3 s rows behind stage 0)
  constexpr int KQ = NS >= 2 ? 3 * (NS - 1) : 1;
  T kq[KQ][V], aq[KQ][V];
  using RowBuf = std::conditional_t<P == kF32, unsigned long long[9], T[9][V]>;
  // The row loop.  The FP32 kernels with three omega = 1 steps (with and
  // without captures) and the FP16S kernel with two (at g = 0) are specialised
  // for strips whose lanes all hold
  // aligned column pairs and store both or neither of their columns (AV, every
  // strip of a lattice whose width is a multiple of the record): their row
  // loads then have no per-lane branch (the compiler had merged the two load
  // shapes into masked branches per population) and they take the uniform
  // stores (store_row) that FP64 takes.  Bitwise the same results; at 4096^2
  // FP32 154.2k -> 157.5k MLUPS (the specialisation alone gained nothing, the
  // uniform stores 2 %), FP16S 164.5k -> 172.3k, the FP32 recompute with
  // captures 156.1 -> 151.6 us per step (its captures uniform too,
  // capture_row).  The other kernels of the two forms would spill with it.
  constexpr bool AV_SPEC = (P == kF32 && W1 && NS == 3 && KF != kGammaKappa) ||
                        (P == kF16S && G0 && W1 && NS == 2 && !CAP && KF != kGammaKappa);
  auto run = [&](auto av) {
    constexpr bool AV = decltype(av)::value;
    constexpr bool UNI = UNI64 || AV;
    RowBuf fa, fb, fc;  // stored values of rows r (being consumed), r + 1 and r + 2
    auto load_buf = [&](rsrc_t row, RowBuf &out) {
      if constexpr (P == kF32) {
        if constexpr (AV) load_row_vec(row, L, out);
        else load_row(row, L, out);
      } else if constexpr (P == kF16S) {
        if constexpr (AV) load_row_vec16(row, L, out);
        else load_row<P>(row, L, out, A);
      } else {
        load_row<P>(row, L, out, A);
      }
    };
    load_buf(rsrc_src(ry), fa);
    if constexpr (KF != kNoField) load_kappa<P, KF>(rsrc_kap(ry), L, ka);
    if (PF >= 2 && KL > 1) {
      const int r1 = (ry + 1) % ny;
      load_buf(rsrc_src(r1), fb);
      if constexpr (KF != kNoField) load_kappa<P, KF>(rsrc_kap(r1), L, kb);
    }
    if (PF == 3 && KL > 2) {
      const int r2 = (ry + 2) % ny;
      load_buf(rsrc_src(r2), fc);
      if constexpr (KF != kNoField) load_kappa<P, KF>(rsrc_kap(r2), L, kc);
    }
    if constexpr (UNI) drop_row_stores<P>(A);  // as a row iteration leaves behind its loads
    if constexpr (P == kF16S) {
      // the c_ly = +1 values of the first row, which fp16s_decode otherwise
      // carries over from the row before
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int i = 0; i < 3; ++i) cn[i][v] = unpack16(fa[2 + i][0], v, A.qinv);
    }

    auto iteration = [&](int k, RowBuf &cur, const RowBuf &nxt, KapBuf<P, KF> &kcur) {
      T f[9][V], f2[9][V];
      if constexpr (P == kF32) {
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          const u32x2 w = __builtin_bit_cast(u32x2, cur[l]);
          const T c[2] = {__uint_as_float(w.x), __uint_as_float(w.y)};
          shift_x<T, V>(l, c, f[l]);
        }
      } else if constexpr (P == kF16S) {
        T d[9][V];
        fp16s_decode<V, G0>(cur, nxt, cs, cq, cn, A, d);
#pragma unroll
        for (int l = 0; l < 9; ++l) shift_x<T, V>(l, d[l], f[l]);
      } else {
#pragma unroll
        for (int l = 0; l < 9; ++l) shift_x<T, V>(l, cur[l], f[l]);
      }
      T k0[V], a0[V];
      if constexpr (KF != kNoField) kappa_cols<P, KF>(kcur, k0, a0);
      S0.ingest(k, f, k0, a0, f2, lane);
      // prefetch row r + PF into the registers just freed.  Past the tile's last
      // row the loads go to an empty buffer range (no memory access, zeros):
      // every iteration issues the same loads, so the compiler's waits for a
      // row need not drain the loads of the rows after it.
      load_buf(k + PF < KL ? rsrc_src(rpre) : make_rsrc(A.src, 0), cur);
      if constexpr (KF != kNoField) load_kappa<P, KF>(k + PF < KL ? rsrc_kap(rpre) : make_rsrc(A.kfield, 0), L, kcur);
      if constexpr (UNI) {
        if (k < KST) drop_row_stores<P>(A);
      }
      T post[9][V], hv[V], jxv[V], jyv[V];
      if (S0.finish(k, f2, post, hv, jxv, jyv, C, L, bad)) {
        const int q = y0 - HALO + k - 2;  // row of the post-collision values (unwrapped)
        if constexpr (NS == 1) {
          store_row<P, G0, UNI>(A, q, post, hv, L, x0, xend, lane);
          if constexpr (CAP) capture_row<P>(A, A.capture, q, hv, jxv, jyv, L, C.href, x0, xend, lane);
        } else {
          const int e = k - 4;  // emission index of stage 0
          if constexpr (CAP) {
            if constexpr (UNI) capture_row<P, true>(A, A.capture, q, hv, jxv, jyv, L, C.href, x0, xend, lane, q >= y0 && q < yend);
            else if (q >= y0 && q < yend) capture_row<P>(A, A.capture, q, hv, jxv, jyv, L, C.href, x0, xend, lane);
          }
          if constexpr (P == kF16S) fp16s_roundtrip<V, G0>(post, hv, A);  // as if stored and reloaded
          T g[9][V];
          H1.feed(post, g);  // row q - 1 of the next step
          if (e >= 2) {
            const int j = e - 2;  // stage 1 row index; its row is q - 1 = y0 - HALO + 3 + j
            T g2[9][V];
            S1.ingest(j, g, kq[2], aq[2], g2, lane);
            T post2[9][V], hv2[V], jx2[V], jy2[V];
            if (S1.finish(j, g2, post2, hv2, jx2, jy2, C, L, bad)) {
              const int q1 = y0 - HALO + 1 + j;  // row of stage 1's post-collision values
              if constexpr (NS == 2) {
                store_row<P, G0, UNI>(A, q1, post2, hv2, L, x0, xend, lane);
                if constexpr (CAP) capture_row<P>(A, A.capture + capblk, q1, hv2, jx2, jy2, L, C.href, x0, xend, lane);
              } else {
                const int e1 = j - 4;  // emission index of stage 1
                if constexpr (CAP) {
                  if constexpr (UNI)
                    capture_row<P, true>(A, A.capture + capblk, q1, hv2, jx2, jy2, L, C.href, x0, xend, lane, q1 >= y0 && q1 < yend);
                  else if (q1 >= y0 && q1 < yend)
                    capture_row<P>(A, A.capture + capblk, q1, hv2, jx2, jy2, L, C.href, x0, xend, lane);
                }
                if constexpr (P == kF16S) fp16s_roundtrip<V, G0>(post2, hv2, A);
                T g3[9][V];
                H2.feed(post2, g3);  // row q1 - 1 of the step after
                if (e1 >= 2) {
                  const int j2 = e1 - 2;  // stage 2 row index; its row is y0 - HALO + 6 + j2
                  T g4[9][V];
                  S2.ingest(j2, g3, kq[KQ - 1], aq[KQ - 1], g4, lane);
                  T post3[9][V], hv3[V], jx3[V], jy3[V];
                  if (S2.finish(j2, g4, post3, hv3, jx3, jy3, C, L, bad)) {
                    const int q2 = y0 - HALO + 4 + j2;
                    store_row<P, G0, UNI>(A, q2, post3, hv3, L, x0, xend, lane);
                    if constexpr (CAP)
                      capture_row<P, UNI>(A, A.capture + 2 * capblk, q2, hv3, jx3, jy3, L, C.href, x0, xend, lane);
                  }
                }
              }
            }
          }
        }
      }
      if constexpr (KF != kNoField && NS >= 2) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
          for (int i = KQ - 1; i > 0; --i) {
            kq[i][v] = kq[i - 1][v];
            if constexpr (KF == kGammaKappa) aq[i][v] = aq[i - 1][v];
          }
          kq[0][v] = k0[v];
          if constexpr (KF == kGammaKappa) aq[0][v] = a0[v];
        }
      }
      ry = ry + 1 == ny ? 0 : ry + 1;
      rpre = rpre + 1 == ny ? 0 : rpre + 1;
    };

    // rows in groups of PF, so that each buffer keeps its registers around the
    // loop; the last rows after it
    int k = 0;
    if constexpr (PF == 3 && UNI) {
      for (; k + 2 < K && k < KST; k += 3) {
        iteration(k, fa, fb, ka);
        iteration(k + 1, fb, fc, kb);
        iteration(k + 2, fc, fa, kc);
      }
      for (; k + 5 < K; k += 6) {
        __builtin_assume(k >= KST);
        iteration(k, fa, fb, ka);
        iteration(k + 1, fb, fc, kb);
        iteration(k + 2, fc, fa, kc);
        iteration(k + 3, fa, fb, ka);
        iteration(k + 4, fb, fc, kb);
        iteration(k + 5, fc, fa, kc);
      }
      for (; k + 2 < K; k += 3) {
        __builtin_assume(k >= KST);
        iteration(k, fa, fb, ka);
        iteration(k + 1, fb, fc, kb);
        iteration(k + 2, fc, fa, kc);
      }
      if (k < K) iteration(k, fa, fb, ka);
      if (k + 1 < K) iteration(k + 1, fb, fc, kb);
    } else if constexpr (PF == 3) {
      // FP16S: groups of six rows (two turns of the three buffers and a whole
      // number of turns of every row history: fewer register moves; +4 % at
      // 4096^2, the form bound by its VALU), then of three.  Not with a
      // surface tension field and captures, where six would spill.
      if constexpr (!(KF == kGammaKappa && CAP)) {
        for (; k + 5 < K; k += 6) {
          iteration(k, fa, fb, ka);
          iteration(k + 1, fb, fc, kb);
          iteration(k + 2, fc, fa, kc);
          iteration(k + 3, fa, fb, ka);
          iteration(k + 4, fb, fc, kb);
          iteration(k + 5, fc, fa, kc);
        }
      }
      for (; k + 2 < K; k += 3) {
        iteration(k, fa, fb, ka);
        iteration(k + 1, fb, fc, kb);
        iteration(k + 2, fc, fa, kc);
      }
      if (k < K) iteration(k, fa, fb, ka);
      if (k + 1 < K) iteration(k + 1, fb, fc, kb);
    } else if constexpr (PF == 2) {
      if constexpr (UNI) {
        // uniform stores: the iterations before KST, then those after, where
        // the compiler is told that every stage stores
        for (; k + 1 < K && k < KST; k += 2) {
          iteration(k, fa, fb, ka);
          iteration(k + 1, fb, fa, kb);
        }
        for (; k + 1 < K; k += 2) {
          __builtin_assume(k >= KST);
          iteration(k, fa, fb, ka);
          iteration(k + 1, fb, fa, kb);
        }
      } else {
        for (; k + 1 < K; k += 2) {
          iteration(k, fa, fb, ka);
          iteration(k + 1, fb, fa, kb);
        }
      }
      if (k < K) iteration(k, fa, fb, ka);
    } else {
      // one row ahead (three steps): FP32 with omega = 1 in groups of six rows,
      // so that the stages' row histories keep their registers (a third fewer
      // moves, +1 %); FP64, the general stages and the surface tension field
      // would need more than 256 VGPRs unrolled
      if constexpr (UNI) {
        // FP32 (without captures) in groups of three rows, a whole turn of the
        // stages' three-row histories, so that they keep their registers
        // (158.8k -> 162.0k MLUPS at 4096^2, bitwise the same); the groups of
        // six of the other branch, and these with captures, would spill
        for (; k < K && k < KST; ++k) iteration(k, fa, fa, ka);
        if constexpr (P == kF32 && !CAP) {
          for (; k + 2 < K; k += 3) {
            __builtin_assume(k >= KST);
            iteration(k, fa, fa, ka);
            iteration(k + 1, fa, fa, ka);
            iteration(k + 2, fa, fa, ka);
          }
        }
        for (; k < K; ++k) {
          __builtin_assume(k >= KST);
          iteration(k, fa, fa, ka);
        }
      } else {
        if constexpr (P == kF32 && W1 && KF != kGammaKappa) {
          for (; k + 5 < K; k += 6) {
            iteration(k, fa, fa, ka);
            iteration(k + 1, fa, fa, ka);
            iteration(k + 2, fa, fa, ka);
            iteration(k + 3, fa, fa, ka);
            iteration(k + 4, fa, fa, ka);
            iteration(k + 5, fa, fa, ka);
          }
        }
        for (; k < K; ++k) iteration(k, fa, fa, ka);
      }
    }
  };
  if constexpr (AV_SPEC) {
    if (L.allvec && L.fast_store) run(std::true_type{});
    else run(std::false_type{});
  } else {
    run(std::false_type{});
  }

  const unsigned long long m = __ballot(bad);
  if (m != 0ull && lane == __ffsll((unsigned long long)m) - 1) atomicOr(A.flag, 1);
}

// ---- launchers -----------------------------------------------------------------
template <int P, int NS, bool G0, int KF, bool W1>
static void launch_step_k(const StepArgs &A, bool cap, hipStream_t s) {
  const dim3 grid(8 * A.per_xcd), block(64);
  if (cap) step_kernel<P, KF, true, NS, G0, W1><<<grid, block, 0, s>>>(A);
  else step_kernel<P, KF, false, NS, G0, W1><<<grid, block, 0, s>>>(A);
}

template <int P, int NS, bool G0, bool W1>
static void launch_step_v(const StepArgs &A, int kf, bool cap, hipStream_t s) {
  if (kf == kGammaKappa) launch_step_k<P, NS, G0, kGammaKappa, W1>(A, cap, s);
  else if (kf == kKappa) launch_step_k<P, NS, G0, kKappa, W1>(A, cap, s);
  else launch_step_k<P, NS, G0, kNoField, W1>(A, cap, s);
}

template <int P, int NS, bool W1>
static hipError_t launch_step_p(const StepArgs &A, int kf, bool cap, hipStream_t s) {
  if constexpr (P == kF16S) {
    if (A.g == 0.0) {
      launch_step_v<P, NS, true, W1>(A, kf, cap, s);
      return hipGetLastError();
    }
  }
  launch_step_v<P, NS, false, W1>(A, kf, cap, s);
  return hipGetLastError();
}

template <int P, bool W1>
static hipError_t launch_step_ns(int ns, const StepArgs &A, int kf, bool cap, hipStream_t s) {
  if constexpr (Form<P>::NSMAX >= 3) {
    if (ns == 3) return launch_step_p<P, 3, W1>(A, kf, cap, s);
  }
  if (ns > 2) return hipErrorInvalidValue;
  if (ns == 2) return launch_step_p<P, 2, W1>(A, kf, cap, s);
  return launch_step_p<P, 1, W1>(A, kf, cap, s);
}

template <int P, int NS, bool G0, bool W1>
static int occupancy_v(int kf) {
  int n = 0;
  const hipError_t e =
      kf == kGammaKappa
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<P, kGammaKappa, false, NS, G0, W1>, 64, 0)
      : kf == kKappa ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<P, kKappa, false, NS, G0, W1>, 64, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<P, kNoField, false, NS, G0, W1>, 64, 0);
  return e == hipSuccess ? n : 0;
}

template <int P, bool W1>
static int occupancy_p(int kf, int ns, bool g0) {
  if constexpr (Form<P>::NSMAX >= 3) {
    if (ns == 3) return occupancy_v<P, 3, false, W1>(kf);
  }
  if (ns > 2) return 0;
  if constexpr (P == kF16S) {
    if (g0) return ns == 2 ? occupancy_v<P, 2, true, W1>(kf) : occupancy_v<P, 1, true, W1>(kf);
  }
  return ns == 2 ? occupancy_v<P, 2, false, W1>(kf) : occupancy_v<P, 1, false, W1>(kf);
}

// Entry points of one storage form and collision stage, each pair defined in
// a translation unit of its own (step_form.hip).
template <int P, bool W1> hipError_t launch_step_form(int ns, const StepArgs &A, int kf, bool cap, hipStream_t s) {
  return launch_step_ns<P, W1>(ns, A, kf, cap, s);
}
template <int P, bool W1> int step_occupancy_form(int kf, int ns, bool g0) { return occupancy_p<P, W1>(kf, ns, g0); }

}  // namespace tflbm
