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

// the same for j known to lie in sets lo .. hi (offsets[lo] <= j < offsets[hi + 1]):
// a workgroup's contiguous chunk of particles spans few sets, so the search
// is usually empty
__device__ __forceinline__ int mock_in(const int64_t* offsets, int lo, int hi, int64_t j) {
  int h = hi + 1;  // offsets[lo] <= j < offsets[h]
  while (h - lo > 1) {
    const int mid = (lo + h) >> 1;
    if (offsets[mid] <= j) lo = mid; else h = mid;
  }
  return lo;
}

template <typename TP>
__device__ __forceinline__ void load_pos(const TP* pos, int64_t j, double& x, double& y, double& z) {
  x = (double)pos[3 * j + 0];
  y = (double)pos[3 * j + 1];
  z = (double)pos[3 * j + 2];
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

// Weights W^(p)(cell - u) of Sec. 2.3 of the p stencil cells along one axis,
// written per offset f = u - floor(u) in [0, 1) for even p and
// f = u - floor(u + 1/2) in [-1/2, 1/2) for odd p (the stencil's first cell
// is floor(...) - (p/2 - 1), resp. - (p-1)/2).
template <int P>
__device__ __forceinline__ void weights_from_offset(float f, float (&w)[P]) {
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
}

// Cells (mod N) and weights of the p-point stencil of one axis, for grid
// coordinate u (float64).  Even p: first cell floor(u) - (p/2 - 1); odd p:
// first cell floor(u + 1/2) - (p-1)/2.
template <int P>
__device__ __forceinline__ void stencil_1d(double u, int n, int (&cell)[P], float (&w)[P]) {
  double fl = (P % 2 == 0) ? floor(u) : floor(u + 0.5);
  const int first = (int)fl - ((P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2);
  weights_from_offset<P>((float)(u - fl), w);
  // first + i lies in [-(p-1), N + p - 1]
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int c = first + i;
    cell[i] = c < 0 ? c + n : (c >= n ? c - n : c);
  }
}

// ---- particle records
// The sort writes one 16-byte record per particle, in bucket order, and the
// deposit reads only these.  Per axis a: the first grid's floor cell c_a
// (floor(u) for even p, floor(u + 1/2) for odd p; mod N), the step s_a from
// it to the same floor on the grid sampled at u + 1/2 (0 or 1), and the
// offset t_a = u - floor(...) (+ 1/2 for odd p), in [0, 1), as a 24-bit
// fraction rounded to nearest: an error of at most 2^-25, that of a float32
// offset in [1/2, 1).  Every cell choice is made on the float64 u.  Words:
//   x: c_x | c_y << 10 | c_z << 20 | s_x << 30 | s_y << 31
//   y: t_x | s_z << 24
//   z: t_y | bits 24..31 free (the two-level sort keeps a bucket index there)
//   w: t_z | bits 24..31 free
constexpr int kFracBits = 24;
constexpr uint32_t kFracMask = (1u << kFracBits) - 1u;

// floor(u) for even p, floor(u + 1/2) for odd p (the record's floor, before
// the reduction mod N)
__device__ __forceinline__ double record_floor(double u, bool even) {
  return even ? floor(u) : floor(u + 0.5);
}

// Bucket of one axis: the bucket of the first grid's first stencil cell
// (record floor minus the stencil offset, mod N).  Keyed this way, the
// particles whose stencil on either grid can reach cells [t0, t0 + T) have
// first cells in [t0 - (p - 1) - 1, t0 + T - 1]: T/4 + ceil(p/4) buckets
// when t0 is a multiple of 4 (keyed by floor(u) it would be T/4 + 2 up to
// p = 4).
__device__ __forceinline__ int bucket_of(double u, const Geom& g) {
  const bool even = (g.order % 2) == 0;
  const int off = even ? g.order / 2 - 1 : (g.order - 1) / 2;
  int f = (int)record_floor(u, even) - off;  // in [-off, N - off]
  f = f < 0 ? f + g.n : (f >= g.n ? f - g.n : f);
  return f / kBucket;
}

__device__ __forceinline__ uint4 particle_record(double ux, double uy, double uz, const Geom& g) {
  const bool even = (g.order % 2) == 0;
  const double u[3] = {ux, uy, uz};
  uint32_t cell[3], step[3], frac[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u2 = u[a] + 0.5;  // the interlaced grid's coordinate
    const double f1 = record_floor(u[a], even);
    const double f2 = record_floor(u2, even);
    const int c1 = (int)f1;  // in [0, N]
    cell[a] = (uint32_t)(c1 >= g.n ? c1 - g.n : c1);
    step[a] = (uint32_t)((int)(f2 - f1) & 1);
    const double t = u[a] - f1 + (even ? 0.0 : 0.5);  // exact, in [0, 1)
    const double q = floor(t * 16777216.0 + 0.5);
    frac[a] = q > 16777215.0 ? kFracMask : (uint32_t)q;
  }
  return make_uint4(cell[0] | (cell[1] << 10) | (cell[2] << 20) | (step[0] << 30) | (step[1] << 31),
                    frac[0] | (step[2] << 24), frac[1], frac[2]);
}

// the offset f (as in weights_from_offset) of one axis from its 24-bit
// fraction t, on the grid sampled at u + 1/2 along this axis when `shifted`:
// there t moves by -1/2 if the floor cell steps, by +1/2 if not (exact)
template <int P>
__device__ __forceinline__ float record_offset(uint32_t t, int step, bool shifted) {
  int q = (int)(t & kFracMask);
  if (shifted) q += step ? -(1 << (kFracBits - 1)) : (1 << (kFracBits - 1));
  float f = (float)q * (1.0f / 16777216.0f);
  if constexpr (P % 2 == 1) f -= 0.5f;
  return f;
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
