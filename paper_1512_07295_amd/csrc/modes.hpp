// Device helpers on Fourier modes shared by the P(k) pass (spectral.hip) and
// the bispectrum (bispec.hip): signed frequencies, shells (Sec. 4 shells of
// width n_dk k_f, decided on integer |m|^2) and the interlace combination of
// eq. intdelta from the transform of rho1 + i rho2.
#pragma once

#include "fft_line.hpp"
#include "fsest_internal.hpp"

namespace fsest {

__device__ __forceinline__ int signed_freq(int i, int n) { return (i <= n / 2) ? i : i - n; }

// -i mod n for 0 <= i < n (a mask when n is a compile-time power of two)
template <bool P2>
__device__ __forceinline__ int neg_mod(int i, int n) {
  if constexpr (P2) return (n - i) & (n - 1);
  else return i ? n - i : 0;
}
// s mod 2n for -2n <= s < 4n: index into the table exp(+i pi s / N)
template <bool P2>
__device__ __forceinline__ int mod_2n(int s, int n) {
  if constexpr (P2) return s & (2 * n - 1);
  else return s < 0 ? s + 2 * n : (s >= 2 * n ? s - 2 * n : s);
}
// FFT index of signed frequency m, |m| < n
__device__ __forceinline__ int fft_index(int m, int n) { return m < 0 ? m + n : m; }

// shell b with (2b-1)^2 n^2 <= 4 m2 < (2b+1)^2 n^2 (b = 0 below the first shell)
__device__ __forceinline__ int shell_of(int m2, int n_dk) {
  const int x = 4 * m2;
  int r = (int)sqrtf((float)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return ((r / n_dk) + 1) >> 1;
}

// Row pair q of one set: rows (x, y) and (-x, -y); q < N^2/2 + 2.
__device__ __forceinline__ void pair_rows(int64_t q, int n, int& x, int& y) {
  const int h1 = n / 2 + 1;
  if (q < h1) { x = 0; y = (int)q; return; }
  q -= h1;
  const int64_t mid = (int64_t)(n / 2 - 1) * n;
  if (q < mid) { x = 1 + (int)(q / n); y = (int)(q % n); return; }
  q -= mid;
  x = n / 2;
  y = (int)q;
}

// Transforms of the real grids at half-space mode (row, mz) from the pair
// (Za, Zb) = (Z(k), Z(-k)), combined per eq. intdelta: returns C(m).
template <bool IL, bool P2 = true>
__device__ __forceinline__ float2 combined_mode(float2 za, float2 zb, int mx, int my, int mz,
                                                const float2* __restrict__ phase, int n) {
  // first and second real transforms: (za + conj zb)/2 and (za - conj zb)/(2i)
  const float2 f1 = make_float2(0.5f * (za.x + zb.x), 0.5f * (za.y - zb.y));
  const float2 f2 = make_float2(0.5f * (za.y + zb.y), 0.5f * (zb.x - za.x));
  if constexpr (IL) {
    const float2 ph = phase[mod_2n<P2>(mx + my + mz, n)];  // exp(+i pi (mx+my+mz)/N)
    return cscale(cadd(f1, cmul(ph, f2)), 0.5f);
  } else {
    // even/odd z samples: F = E + exp(-2 pi i mz/N) O
    const float2 ph = cconj(phase[mod_2n<P2>(2 * mz, n)]);
    return cadd(f1, cmul(ph, f2));
  }
}

// |K C(m)|^2 from the pair (Za, Zb) = (Z(k), Z(-k)) and the phase ph of
// combined_mode: with a = Za, b = conj(Zb), 2 F1 = a + b and 2 F2 = (a - b)/i,
// so (cx, cy) = 2 (F1 + ph F2).  The interlaced combination is
// C = (F1 + ph F2)/2 (K = 4); the packed real grid's is C = F1 + ph F2 (K = 2).
__device__ __forceinline__ float pair_power(float2 za, float2 zb, float2 ph) {
  const float sx = za.x + zb.x, sy = za.y - zb.y;
  const float dx = za.x - zb.x, dy = za.y + zb.y;
  const float cx = sx + (ph.x * dy + ph.y * dx);
  const float cy = sy + (ph.y * dy - ph.x * dx);
  return cx * cx + cy * cy;
}

// C(m) of interlacing codes 2 and 3 (more than two grids): C = (1/G) sum_j
// F_j(m) exp(+i pi s_j / N), s_j the sum of the components of m along the
// axes grid j is shifted on, with F_2q and F_2q+1 unpacked from slab q's
// Z(k) and Z(-k) as in combined_mode.  Signed m, |m_a| <= N/2.
__device__ __forceinline__ float2 multi_mode(const float2* __restrict__ data, const Geom& g,
                                             int mock, int mx, int my, int mz,
                                             const float2* __restrict__ phase) {
  const int n = g.n;
  const int x = fft_index(mx, n), y = fft_index(my, n), z = fft_index(mz, n);
  const int xm = neg_mod<false>(x, n), ym = neg_mod<false>(y, n), zm = neg_mod<false>(z, n);
  const int m[3] = {mx, my, mz};
  float2 c = make_float2(0.f, 0.f);
  for (int q = 0; q < g.npair; ++q) {
    const int slab = mock * g.npair + q;
    const float2 za = data[complex_index(g, slab, x, y, z)];
    const float2 zb = data[complex_index(g, slab, xm, ym, zm)];
    const float2 f[2] = {make_float2(0.5f * (za.x + zb.x), 0.5f * (za.y - zb.y)),
                         make_float2(0.5f * (za.y + zb.y), 0.5f * (zb.x - za.x))};
    for (int h = 0; h < 2; ++h) {
      const int mk = grid_mask(g.code, 2 * q + h);
      int sj = 0;
      for (int a = 0; a < 3; ++a) sj += ((mk >> a) & 1) ? m[a] : 0;
      c = cadd(c, cmul(phase[mod_2n<false>(sj, n)], f[h]));
    }
  }
  return cscale(c, 1.0f / (float)g.ng);
}

}  // namespace fsest
