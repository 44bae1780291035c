// Device-side building blocks shared by the forward and reverse kernels of
// the thin-film lattice Boltzmann step (arXiv:1810.07642, Sec. II).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tflbm {

enum Prec { kF64 = 0, kF32 = 1, kF16S = 2 };

// D2Q9 velocities, l = 0..8 counter-clockwise from +x; odd l on the axes,
// even l on the diagonals (Sec. II, eq. "speeds").
constexpr int kCx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kCy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
// Weights (Sec. II).
constexpr double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0,
                          1.0 / 9.0, 1.0 / 36.0, 1.0 / 9.0, 1.0 / 36.0};
constexpr double kCs2 = 1.0 / 3.0;

// Storage form of the populations.
//  V  : consecutive columns owned by one lane of a marching wavefront.
//  T  : arithmetic type of the step.
template <int P> struct Form;
template <> struct Form<kF64> { using T = double; static constexpr int V = 1; };
template <> struct Form<kF32> { using T = float; static constexpr int V = 2; };
template <> struct Form<kF16S> { using T = float; static constexpr int V = 2; };

// Everything a step kernel needs, passed by value.
struct StepArgs {
  const char *src;        // populations at time t (push layout: f_l(x) at x)
  char *dst;              // populations at time t + 1
  const void *kfield;     // kappa field [ny][ldx] in T, or nullptr for kappa0
  char *capture;          // h, jx, jy planes [3][ny][ldx] in T, or nullptr
  int *flag;              // status word: bit 0 set on h <= 0 or non-finite h
  int nx, ny, ldx;
  int64_t plane;          // ny * ldx elements
  int nstrips, H, ntiles, per_xcd;
  int n_exp, m_exp;
  double omega, gamma, nu, hstar, delta, ax, ay, g, kappa0;
  double shift[9];        // FP16S: rest-equilibrium shift of each moving population
  float qscale, qinv;     // FP16S: 2^s and 2^-s
};

__device__ __forceinline__ int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Value of `v` held by lane - 1 (own value on lane 0) / lane + 1 (own value on lane 63).
template <typename T> __device__ __forceinline__ T from_left(T v) { return __shfl_up(v, 1); }
template <typename T> __device__ __forceinline__ T from_right(T v) { return __shfl_down(v, 1); }

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

// ---- population storage -------------------------------------------------
// Plane l of a buffer: FP64/FP32 planes of T; FP16S: plane 0 FP32, planes
// 1..8 FP16 stored after it.
template <int P> __device__ __forceinline__ size_t plane_offset(int l, int64_t plane) {
  if constexpr (P == kF64) return (size_t)l * plane * 8;
  else if constexpr (P == kF32) return (size_t)l * plane * 4;
  else return l == 0 ? 0 : (size_t)plane * 4 + (size_t)(l - 1) * plane * 2;
}

template <int P> struct Pop;

template <> struct Pop<kF64> {
  __device__ static void load(const char *buf, int l, const StepArgs &A, int row, const int *col,
                              bool /*vec*/, double *out) {
    const double *p = (const double *)(buf + plane_offset<kF64>(l, A.plane)) + (size_t)row * A.ldx;
    out[0] = p[col[0]];
  }
};

template <> struct Pop<kF32> {
  __device__ static void load(const char *buf, int l, const StepArgs &A, int row, const int *col,
                              bool vec, float *out) {
    const float *p = (const float *)(buf + plane_offset<kF32>(l, A.plane)) + (size_t)row * A.ldx;
    if (vec) {
      float2 v = *(const float2 *)(p + col[0]);
      out[0] = v.x;
      out[1] = v.y;
    } else {
      out[0] = p[col[0]];
      out[1] = p[col[1]];
    }
  }
};

template <> struct Pop<kF16S> {
  __device__ static void load(const char *buf, int l, const StepArgs &A, int row, const int *col,
                              bool vec, float *out) {
    if (l == 0) {
      const float *p = (const float *)buf + (size_t)row * A.ldx;
      if (vec) {
        float2 v = *(const float2 *)(p + col[0]);
        out[0] = v.x;
        out[1] = v.y;
      } else {
        out[0] = p[col[0]];
        out[1] = p[col[1]];
      }
    } else {
      const __half *p = (const __half *)(buf + plane_offset<kF16S>(l, A.plane)) + (size_t)row * A.ldx;
      float s = (float)A.shift[l];
      if (vec) {
        __half2 v = *(const __half2 *)(p + col[0]);
        out[0] = s + __low2float(v) * A.qinv;
        out[1] = s + __high2float(v) * A.qinv;
      } else {
        out[0] = s + __half2float(p[col[0]]) * A.qinv;
        out[1] = s + __half2float(p[col[1]]) * A.qinv;
      }
    }
  }
};

}  // namespace tflbm
