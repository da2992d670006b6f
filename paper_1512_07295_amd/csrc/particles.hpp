// Device helpers shared by the sort, the deposit and the adjoint gather:
// particle lookup, cell location and the order-p stencils (Sec. 2.3).
#pragma once

#include "fsest_internal.hpp"

namespace fsest {

// mass of particle j divided by the largest mass (in [0, 1]; 0 if every mass is 0)
__device__ __forceinline__ float scaled_mass(const float* w, int64_t j, const uint32_t* stats) {
  const float wmax = __uint_as_float(stats[4]);
  const float v = w[j];
  return (wmax > 0.0f && v >= 0.0f && v <= wmax) ? v / wmax : 0.0f;
}

// set index of particle j: largest i with offsets[i] <= j (offsets has batch+1 entries)
__device__ __forceinline__ int mock_of(const int64_t* offsets, int batch, int64_t j) {
  if (batch == 1 || offsets == nullptr) return 0;
  int lo = 0, hi = batch;  // offsets[lo] <= j < offsets[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (offsets[mid] <= j) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename TP>
__device__ __forceinline__ void load_pos(const TP* pos, int64_t j, double& x, double& y, double& z) {
  x = (double)pos[3 * j + 0];
  y = (double)pos[3 * j + 1];
  z = (double)pos[3 * j + 2];
}

// floor(u) mod N for u in [0, N] (u = N can come out of the rounding of x N / L)
__device__ __forceinline__ int base_cell(double u, int n) {
  const int c = (int)floor(u);
  return c >= n ? c - n : c;
}

// ------------------------------------------------------------------ stencils
// Orders above 4 (the higher-order B-splines of Sec. 2.3): the weights of
// the p stencil cells are N_p(t + i), i = 0..p-1, of the cardinal B-spline
// N_p (the p-fold convolution of the unit box on [0, 1], support [0, p]),
// with t = 1 - f for even p and t = 1/2 - f for odd p (f = u - floor(...)
// as below), from the recursion
//   N_{k+1}(t + j) = ((t + j) N_k(t + j) + (k + 1 - t - j) N_k(t + j - 1)) / k,
// N_1(t) = 1 (convex combinations: no cancellation).  d/ds of the order-p
// weight is N_{p-1}(t + i) - N_{p-1}(t + i - 1), from the previous level.
template <int P>
__device__ __forceinline__ void bspline_weights(float t, float (&w)[P], float (&wd)[P]) {
  float v[P];
#pragma unroll
  for (int j = 0; j < P; ++j) v[j] = (j == 0) ? 1.0f : 0.0f;
#pragma unroll
  for (int k = 1; k < P; ++k) {
    if (k == P - 1) {
#pragma unroll
      for (int j = 0; j < P; ++j) wd[j] = (j < k ? v[j] : 0.0f) - (j >= 1 ? v[j - 1] : 0.0f);
    }
    float nv[P];
    const float rk = 1.0f / (float)k;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const float a = (j < k) ? v[j] : 0.0f;
      const float b = (j >= 1 && j <= k) ? v[j - 1] : 0.0f;
      nv[j] = (j <= k) ? ((t + (float)j) * a + ((float)(k + 1 - j) - t) * b) * rk : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = nv[j];
  }
#pragma unroll
  for (int j = 0; j < P; ++j) w[j] = v[j];
}

// Cells (mod N) and weights of the p-point stencil of one axis, for grid
// coordinate u (float64).  Even p: first cell floor(u) - (p/2 - 1); odd p:
// first cell floor(u + 1/2) - (p-1)/2.  Weights are W^(p)(cell - u) of
// Sec. 2.3 written per offset with f = u - floor(...).
template <int P>
__device__ __forceinline__ void stencil_1d(double u, int n, int (&cell)[P], float (&w)[P]) {
  double fl = (P % 2 == 0) ? floor(u) : floor(u + 0.5);
  const int first = (int)fl - ((P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2);
  const float f = (float)(u - fl);
  if constexpr (P == 1) {
    w[0] = 1.0f;
  } else if constexpr (P == 2) {
    w[0] = 1.0f - f;
    w[1] = f;
  } else if constexpr (P == 3) {
    const float a = 0.5f - f, c = 0.5f + f;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - f * f;
    w[2] = 0.5f * c * c;
  } else if constexpr (P == 4) {
    const float t = 1.0f - f;
    const float f2 = f * f, t2 = t * t;
    w[0] = t2 * t * (1.0f / 6.0f);
    w[1] = (4.0f - 6.0f * f2 + 3.0f * f2 * f) * (1.0f / 6.0f);
    w[2] = (4.0f - 6.0f * t2 + 3.0f * t2 * t) * (1.0f / 6.0f);
    w[3] = f2 * f * (1.0f / 6.0f);
  } else {
    float wd[P];
    bspline_weights<P>((P % 2 == 0) ? 1.0f - f : 0.5f - f, w, wd);
  }
  // first + i lies in [-(p-1), N + p - 1]
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int c = first + i;
    cell[i] = c < 0 ? c + n : (c >= n ? c - n : c);
  }
}

// derivative dW/ds of the same weights (s = cell - u)
template <int P>
__device__ __forceinline__ void stencil_1d_deriv(double u, float (&dw)[P]) {
  double fl = (P % 2 == 0) ? floor(u) : floor(u + 0.5);
  const float f = (float)(u - fl);
  if constexpr (P == 1) {
    dw[0] = 0.0f;
  } else if constexpr (P == 2) {
    // s = -f (|s|<1, s<=0) -> W' = +1 ; s = 1-f > 0 -> W' = -1
    // at f == 0: s = 0 gives sign(0) = 0 and s = 1 lies outside |s| < 1
    dw[0] = (f > 0.0f) ? 1.0f : 0.0f;
    dw[1] = (f > 0.0f) ? -1.0f : 0.0f;
  } else if constexpr (P == 3) {
    // s0 = -1-f, s1 = -f, s2 = 1-f
    dw[0] = (0.5f - f);           // W' = -(3/2-|s|) sgn(s), s<0 -> +(1/2 - f)
    dw[1] = 2.0f * f;             // -2 s
    dw[2] = -(0.5f + f);          // s>0 -> -(3/2 - (1-f))
  } else if constexpr (P > 4) {
    float w[P];
    bspline_weights<P>((P % 2 == 0) ? 1.0f - f : 0.5f - f, w, dw);
  } else {
    const float t = 1.0f - f;
    // s0 = -1-f (|s| in [1,2)): W' = +(1/2)(2-|s|)^2 = t^2/2
    dw[0] = 0.5f * t * t;
    // s1 = -f: W' = -2 s + 1.5 s |s| = 2 f - 1.5 f^2
    dw[1] = 2.0f * f - 1.5f * f * f;
    // s2 = 1 - f = t: W' = -2 t + 1.5 t^2
    dw[2] = -2.0f * t + 1.5f * t * t;
    // s3 = 2 - f (|s| in (1,2]): W' = -(1/2)(2-|s|)^2 = -f^2/2
    dw[3] = -0.5f * f * f;
  }
}

}  // namespace fsest
