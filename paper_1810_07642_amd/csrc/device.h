// Device-side building blocks shared by the forward and reverse kernels of
// the thin-film lattice Boltzmann step (arXiv:1810.07642, Sec. II).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tflbm {

enum Prec { kF64 = 0, kF32 = 1, kF16S = 2 };

// Per-site field the film pressure reads: none (uniform kappa0 and gamma),
// kappa [ny][ldx], or, for a position-dependent surface tension, the pair
// (-gamma/6, -gamma kappa) per site [ny][ldx][2] (p = -gamma (lap h + kappa phi)).
enum FieldKind { kNoField = 0, kKappa = 1, kGammaKappa = 2 };

// D2Q9 velocities, l = 0..8 counter-clockwise from +x; odd l on the axes,
// even l on the diagonals (Sec. II, eq. "speeds").
constexpr int kCx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kCy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
// Weights (Sec. II).
constexpr double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0,
                          1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0};
constexpr double kCs2 = 1.0 / 3.0;

// Storage form of the populations.
//  V   : consecutive columns owned by one lane of a marching wavefront.
//  T   : arithmetic type of the step.
//  B   : sites per record (one marching strip writes exactly one record per
//        row).  A wavefront covers 64 V columns: B output columns and
//        HX = (64 V - B)/2 halo columns per side; NS fused steps consume
//        3 NS of them (the stencil reaches 3 columns per step).  With V = 2
//        HX is even, so that every lane's column pair is 8-byte aligned.
//  NSMAX: the most fused steps per pass the halo allows (three only with the
//        omega = 1 stage, whose history lives in registers; the general
//        stage keeps two rows of nine populations per step in LDS, and three
//        of those cap a CU at five wavefronts).
//  RB  : bytes per record.
//  Each c_ly group of segments is padded to whole 128-byte lines and the
//  step writes the padding too, so every line of a full record is written
//  whole (pad_offset, pad_bytes).
constexpr int lines128(int bytes) { return (bytes + 127) / 128 * 128; }
template <int P> struct Form;
template <> struct Form<kF64> {
  // segments of 368 B; groups of three padded from 1104 to 1152 B (9 lines);
  // 27 lines per record, an odd stride over the HBM channels.  Nine halo
  // columns: three fused steps.  (52-site records with six halo columns, the
  // most two steps need, ran two steps per pass 5 % faster, 58.0k against
  // 54.9k MLUPS at 4096^2; three omega = 1 steps on 46-site records run at
  // 70k.)
  using T = double;
  static constexpr int V = 1, B = 46, SEG = B * 8, GRP = lines128(3 * SEG), RB = 3 * GRP, NSMAX = 3;
};
template <> struct Form<kF32> {
  // segments of 432 B; groups of three padded from 1296 to 1408 B (11 lines);
  // 33 lines per record, an odd stride over the HBM channels.  Ten halo
  // columns (nine for three steps, rounded up to keep every lane's column
  // pair 8-byte aligned): three fused steps.  Two steps per pass run as fast
  // as on 116-site records (115k MLUPS at 4096^2).
  using T = float;
  static constexpr int V = 2, B = 108, SEG = B * 4, GRP = lines128(3 * SEG), RB = 3 * GRP, NSMAX = 3;
};
template <> struct Form<kF16S> {
  // source height deviation FP32 (464 B) and 8 FP16 segments of 232 B; the
  // c_ly groups start on lines: {s, slots 1-2} at 0 (1024 B), slots 3-5 at G1
  // (768 B), slots 6-8 at G2 (768 B), plus one unused line: 21 lines, an odd
  // stride (a power-of-two record stride puts the same segment of every
  // record on the same few HBM channels).  At most two fused steps: FP16S
  // is bound by its VALU, which a third step (narrower records, more halo
  // work per output) does not relieve (three with the LDS history: 97k
  // against 143k MLUPS at 4096^2)
  using T = float;
  static constexpr int V = 2, B = 116, SEG = B * 2, NSMAX = 2;
  static constexpr int G1 = lines128(4 * B + 2 * SEG), G2 = G1 + lines128(3 * SEG);
  static constexpr int RB0 = G2 + lines128(3 * SEG);
  static constexpr int RB = (RB0 / 128) % 2 ? RB0 : RB0 + 128;
};

// Population layout ("pull in x, push in y").  Records of B consecutive
// columns of one row, [ny][ceil(nx/B)][record].  Population l of site (x, y)
// is stored in row y at column x - c_lx (periodic): the post-collision value
// of site (x, y) is written at column x of row y + c_ly, so every lane stores
// its own columns, and the x shift of streaming is taken on the read side.
// Inside a record the nine segments are ordered by c_ly (0, +1, -1), so the
// populations a row writes into each of its three destination rows are
// contiguous.
constexpr int kSlot[9] = {0, 1, 3, 4, 5, 2, 6, 7, 8};

// Byte offset of the segment of population l inside a record.
template <int P> __host__ __device__ constexpr int seg_offset(int l) {
  if constexpr (P == kF64 || P == kF32) {
    return (kSlot[l] / 3) * Form<P>::GRP + (kSlot[l] % 3) * Form<P>::SEG;
  } else {
    // FP16S: site height deviation FP32 at 0, FP16 slots 1-2 after it, slots
    // 3-5 at G1, slots 6-8 at G2 (each c_ly group starts on a 128-byte line)
    using F = Form<kF16S>;
    constexpr int S = F::SEG;
    const int s = kSlot[l];
    return s == 0 ? 0 : (s <= 2 ? 4 * F::B + (s - 1) * S : (s <= 5 ? F::G1 + (s - 3) * S : F::G2 + (s - 6) * S));
  }
}

// Capture of one step (the moments h, h u_x, h u_y of the pre-collision state,
// for the reverse sweep): records of the same B columns, [ny][ceil(nx/B)]
// [record], each holding the three B-element segments of the working type and
// padded to whole 128-byte lines, so the step writes whole lines.
template <int P> __host__ __device__ constexpr int cap_record_bytes() {
  return (3 * Form<P>::B * (int)sizeof(typename Form<P>::T) + 127) / 128 * 128;
}

// Byte offset and size of the padding after c_ly group g (0: c_ly = 0,
// 1: +1, 2: -1).
template <int P> __host__ __device__ constexpr int pad_offset(int g) {
  if constexpr (P == kF64 || P == kF32) return g * Form<P>::GRP + 3 * Form<P>::SEG;
  else return g == 0 ? 4 * Form<kF16S>::B + 2 * Form<kF16S>::SEG
                     : (g == 1 ? Form<kF16S>::G1 : Form<kF16S>::G2) + 3 * Form<kF16S>::SEG;
}
template <int P> __host__ __device__ constexpr int pad_bytes(int g) {
  if constexpr (P == kF64 || P == kF32) return Form<P>::GRP - 3 * Form<P>::SEG;
  else return g == 0 ? Form<kF16S>::G1 - 4 * Form<kF16S>::B - 2 * Form<kF16S>::SEG
                     : Form<kF16S>::G2 - Form<kF16S>::G1 - 3 * Form<kF16S>::SEG;
}
static_assert(Form<kF16S>::RB0 - Form<kF16S>::G2 == Form<kF16S>::G2 - Form<kF16S>::G1,
              "the c_ly = +1 and -1 groups of an FP16S record have the same padded size");

// Everything a step kernel needs, passed by value.
struct StepArgs {
  const char *src;        // population records at time t
  char *dst;              // population records at time t + 1
  const void *kfield;     // per-site field (FieldKind: kappa [ny][ldx] or pairs [ny][ldx][2] in T), or nullptr
  char *capture;          // h, jx, jy planes [3][ny][ldx] in T, or nullptr
  int *flag;              // status word: bit 0 set on h <= 0 or non-finite h
  int nx, ny, ldx;        // ldx: pitch of the plane arrays (kappa, capture)
  int64_t plane;          // ny * ldx elements
  int nblk;               // records per row, ceil(nx / B)
  int nstrips, H, ntiles, per_xcd;
  int n_exp, m_exp;
  double omega, gamma, nu, hstar, delta, ax, ay, g, kappa0;
  double href;            // reference height: stored d_l = f_l - E_l(href), h = href + sum d
  float qscale, qinv;     // FP16S: 2^s and 2^-s
};

// ---- buffer access ----------------------------------------------------------
// Raw buffer loads/stores: a wave-uniform resource (base address and byte
// length, held in scalar registers) and a per-lane 32-bit byte offset, so the
// hot loop spends no vector instructions on 64-bit address arithmetic.
// Offsets at or beyond the length read 0 and drop stores.
// Cache policies (the last operand): loads keep the default, so that the halo
// rows and columns a tile re-reads can still hit in L2; stores are
// non-temporal (the streaming hint, bit 1), as every stored byte is read
// back only by the next pass.  Measured at 4096^2: non-temporal stores gain
// 1-2 % in every storage form, non-temporal loads lose 14-22 %.
constexpr int kLoadPolicy = 0, kStorePolicy = 2;
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float ld_f32(rsrc_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadPolicy));
}
__device__ __forceinline__ float2 ld_f32x2(rsrc_t r, int off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kLoadPolicy));
}
__device__ __forceinline__ double ld_f64(rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kLoadPolicy));
}
__device__ __forceinline__ __half ld_f16(rsrc_t r, int off) {
  return __ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, kLoadPolicy));
}
__device__ __forceinline__ __half2 ld_f16x2(rsrc_t r, int off) {
  return __builtin_bit_cast(__half2, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kLoadPolicy));
}
__device__ __forceinline__ void st_f32(rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, kStorePolicy);
}
__device__ __forceinline__ void st_f32x2(rsrc_t r, int off, float a, float b) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, make_float2(a, b)), r, off, 0, kStorePolicy);
}
__device__ __forceinline__ void st_f64(rsrc_t r, int off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStorePolicy);
}
__device__ __forceinline__ void st_f16(rsrc_t r, int off, __half v) {
  __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(v), r, off, 0, kStorePolicy);
}
__device__ __forceinline__ void st_f16x2(rsrc_t r, int off, __half a, __half b) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, __halves2half2(a, b)), r, off, 0, kStorePolicy);
}
__device__ __forceinline__ void st_t(rsrc_t r, int off, float v) { st_f32(r, off, v); }
__device__ __forceinline__ void st_t(rsrc_t r, int off, double v) { st_f64(r, off, v); }

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Decoded FP16S deviation q * 2^-s.  Written as a fused multiply-add with a
// zero addend (the same rounded product) so that the conversion and the
// scaling can issue as one mixed-precision instruction.
__device__ __forceinline__ float dec16(__half q, float qinv) { return __builtin_fmaf(__half2float(q), qinv, 0.0f); }

// Value of `v` held by lane - 1 (0 on lane 0) / lane + 1 (0 on lane 63): DPP
// whole-wavefront shifts by one lane (wave_shr:1 = 0x138, wave_shl:1 =
// 0x130).  A lane without a source reads zero (bound_ctrl), which lets the
// compiler fold the shift into the instruction that consumes it instead of
// a move of its own plus a copy of the old value; the end lanes of a
// wavefront are halo, whose values no stored column depends on.  Measured
// at 4096^2: FP16S +1.3 % MLUPS, the FP64 reverse pass -2.7 % time, outputs
// bit for bit unchanged.
__device__ __forceinline__ int wave_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int wave_shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(wave_shr1(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(wave_shl1(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = wave_shr1((int)(b & 0xffffffffll)), hi = wave_shr1((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = wave_shl1((int)(b & 0xffffffffll)), hi = wave_shl1((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// a * b + c, fused (one rounding) in both precisions.  The FP64 step once kept
// two roundings, as its unfused reference does; fused it is 3 % faster at
// 4096^2 (82.3k -> 84.9k MLUPS on one box) and as close to the FP64 oracle
// (every parity test within its 1e-12).  Nothing else is contracted
// (-ffp-contract=off).
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double madd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x: the hardware reciprocal (about 1 ulp) in FP32; in FP64 the hardware
// estimate refined by two Newton-Raphson steps, r <- r + r (1 - x r), each an
// FMA pair (within about an ulp for the film heights and friction
// denominators it serves, which are normal numbers far from the range ends).
// The correctly rounded quotient costs about eleven instructions against five
// (scaling, a correction step and the final fix-up); with three reciprocals
// per site and step the FP64 step ran 4.9 % faster at 4096^2 (75.7k -> 79.4k
// MLUPS on one box), and stays within 1e-12 of the FP64 oracle.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// (h_*/h)^n - (h_*/h)^m given r = h_*/h; (9, 3) and (3, 9) without loops.
template <typename T> __device__ __forceinline__ T ipow(T x, int n);
template <typename T> __device__ __forceinline__ T disjoining(T r, int n, int m) {
  if ((n == 9 && m == 3) || (n == 3 && m == 9)) {
    const T r3 = r * r * r;
    const T r9 = r3 * r3 * r3;
    return n == 9 ? r9 - r3 : r3 - r9;
  }
  return ipow(r, n) - ipow(r, m);
}

// x^n for a small non-negative integer n by repeated squaring.
template <typename T> __device__ __forceinline__ T ipow(T x, int n) {
  T r = T(1);
  T b = x;
  while (n > 0) {
    if (n & 1) r *= b;
    b *= b;
    n >>= 1;
  }
  return r;
}

// ---- population storage ------------------------------------------------
// FP16S keeps, per stored site, the height deviation s of the site whose
// c_ly = 0 populations it holds (its source: the site itself) in FP32, and
// each moving population as the FP16 difference from the rest equilibrium of
// its own source (Sec. II, eq. "equilibria" at u = 0):
//   q_l = (d_l - e_l(s_src)) 2^scale,  e_l(s) = E_l(href + s) - E_l(href),
// i.e. g s (s + 2 href)/6 on the axes and /24 on the diagonals.  In the
// "pull in x, push in y" records the entry of population l at (column X,
// row Y) came from site (X, Y - c_ly), so s_src sits in the same column one
// row up (c_ly = +1), in the same row (0) or one row down (-1).  The rest
// deviation is implicit: d_0 = s - sum_{l>=1} (e_l(s) + q_l 2^-scale) over
// the site's own moving populations (stored at (X, Y + c_ly)), summed in the
// order l = 1..8, so a site's nine values add up to s and the total mass is
// the sum of the stored s.  Encoding and decoding below use the same
// expressions, so a value decoded from memory equals the one the writer
// formed.
struct Rest16 {
  float ax, dg;
};
__device__ __forceinline__ Rest16 rest16(float s, float g, float two_href) {
  const float G = (g * s) * (s + two_href);
  return {G * (1.0f / 6.0f), G * (1.0f / 24.0f)};
}
__device__ __forceinline__ float rest16_l(const Rest16 &e, int l) { return (l & 1) ? e.ax : e.dg; }
// d_0 of a site from its s and the decoded moving populations it emitted.
__device__ __forceinline__ float rest16_d0(float s, const float (&d)[9]) {
  float t = s;
#pragma unroll
  for (int l = 1; l < 9; ++l) t -= d[l];
  return t;
}

// FP16S: the stored height deviation s of the site at (row y, column c).
__device__ __forceinline__ float src16_at(const char *buf, int y, int c, const StepArgs &A) {
  constexpr int B = Form<kF16S>::B;
  const int blk = c / B, pos = c - blk * B;
  return ((const float *)(buf + ((size_t)y * A.nblk + blk) * Form<kF16S>::RB))[pos];
}

// Stored deviation d_l = f_l - E_l(href) of population l at (row y, stored
// column c), widened to T.
template <int P>
__device__ __forceinline__ typename Form<P>::T pop_at(const char *buf, int l, int y, int c, const StepArgs &A) {
  constexpr int B = Form<P>::B;
  const int blk = c / B, pos = c - blk * B;
  auto rec = [&](int row, int m) {
    return buf + ((size_t)row * A.nblk + blk) * Form<P>::RB + seg_offset<P>(m);
  };
  if constexpr (P == kF64) return ((const double *)rec(y, l))[pos];
  else if constexpr (P == kF32) return ((const float *)rec(y, l))[pos];
  else {
    const float g = (float)A.g, h2 = 2.0f * (float)A.href;
    const bool g0 = A.g == 0.0;  // as in the step: no rest-equilibrium part to add
    if (l != 0) {
      const float q = dec16(((const __half *)rec(y, l))[pos], A.qinv);
      if (g0) return q;
      const int ys = wrap(y - kCy[l], A.ny);
      const Rest16 e = rest16(((const float *)rec(ys, 0))[pos], g, h2);
      return rest16_l(e, l) + q;
    }
    const float s0 = ((const float *)rec(y, 0))[pos];
    const Rest16 e = rest16(s0, g, h2);
    float d[9];
    d[0] = 0.0f;
#pragma unroll
    for (int m = 1; m < 9; ++m) {
      const float q = dec16(((const __half *)rec(wrap(y + kCy[m], A.ny), m))[pos], A.qinv);
      d[m] = g0 ? q : rest16_l(e, m) + q;
    }
    return rest16_d0(s0, d);
  }
}

}  // namespace tflbm
