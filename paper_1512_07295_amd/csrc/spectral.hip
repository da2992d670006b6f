// Fourier-space stages: interlacing (eq. intdelta), window deconvolution
// (eqs. windowcorrection, intkerFT), |k|-shell sums for P(k) (eq. ps and the
// estimator of Sec. 2.2) and the adjoint spectrum.  The bispectrum is in
// bispec.hip.
//
// The grid holds Z = FFT(rho1 + i rho2) (interlaced) or Z = FFT of the real
// grid packed pairwise along z (h = N/2 complex columns).  Either way the
// transforms of the real grids at m need Z(m) and Z(-m) together, so the last
// axis is processed by pairs of rows (x, y) and (-x, -y): a workgroup runs
// the z FFT of both rows, keeps them in LDS and finishes every half-space mode
// of the pair without writing the spectrum back.
#include "fft_line.hpp"
#include "modes.hpp"

namespace fsest {

// ------------------------------------------------------------------ tables
__global__ void k_tables(Geom g, float2* tw_n, float2* tw_nz, float* inv_w2, float* win1,
                         float2* phase) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (i < n) {
    double s, c;
    sincospi(-2.0 * i / n, &s, &c);
    tw_n[i] = make_float2((float)c, (float)s);
    const int m = (i <= n / 2) ? i : i - n;
    double w = 1.0;
    if (m != 0) {
      const double x = (double)m / n;
      w = sinpi(x) / (M_PI * x);
    }
    double wp = 1.0;
    for (int k = 0; k < g.order; ++k) wp *= w;
    win1[i] = (float)wp;
    inv_w2[i] = (float)(1.0 / (wp * wp));
  }
  if (i < g.nz) {
    double s, c;
    sincospi(-2.0 * i / g.nz, &s, &c);
    tw_nz[i] = make_float2((float)c, (float)s);
  }
  if (i < 2 * n) {
    double s, c;
    sincospi((double)i / n, &s, &c);
    phase[i] = make_float2((float)c, (float)s);
  }
}

hipError_t launch_tables(const Geom& g, const Buffers& b, hipStream_t s) {
  const int n = 2 * g.n;
  hipLaunchKernelGGL(k_tables, dim3((n + 255) / 256), dim3(256), 0, s, g, b.tw_n, b.tw_nz,
                     b.inv_w2, b.win1, b.phase);
  return hipGetLastError();
}

template <int L>
struct PairShape {
  static constexpr int TPL = LinePlan<L>::TPL;
  static constexpr int PPB = (256 / (2 * TPL)) > 0 ? (256 / (2 * TPL)) : 1;
  static constexpr int THREADS = PPB * 2 * TPL;
  static constexpr int ROWP = LdsLine<L>::padded;
  static constexpr int EPT = LinePlan<L>::EPT;
  static constexpr int ROWS_LDS = 2 * PPB * ROWP;
};
// L = 0: row length 2^a 3^b 5^c with a run-time plan (tpl = ceil(L/16)
// threads per row, 16 elements per thread); PPB = max(1, 128 / tpl) pairs,
// so 2 PPB (L + L/16 + 1) <= 4608 elements as for the FFT rows
template <>
struct PairShape<0> {
  static constexpr int THREADS = 256;
  static constexpr int EPT = 16;
  static constexpr int ROWS_LDS = 4608;
};
__host__ __device__ inline int rt_pairs_per_block(int tpl) { return 128 / tpl > 0 ? 128 / tpl : 1; }

// MODE 0: forward z FFT + P(k) shell sums; MODE 1: shell sums of a stored
// spectrum; MODE 2: forward z FFT, adjoint spectrum, inverse z FFT, write.
template <int L, bool IL, int MODE>
__global__ __launch_bounds__(PairShape<L>::THREADS) void k_pairs(
    float2* __restrict__ data, Geom g, const float2* __restrict__ tw,
    const float2* __restrict__ phase, const float* __restrict__ inv_w2, int n_dk, int n_bins,
    double* __restrict__ partials, const double* __restrict__ coef, RtLine rt) {
  constexpr bool P2 = L != 0;  // compile-time power-of-two row length
  constexpr int EPT = PairShape<L>::EPT;
  int TPL, PPB, ROWP, LL;
  if constexpr (P2) {
    TPL = PairShape<L>::TPL;
    PPB = PairShape<L>::PPB;
    ROWP = PairShape<L>::ROWP;
    LL = L;
  } else {
    TPL = rt.tpl;
    PPB = rt_pairs_per_block(rt.tpl);
    ROWP = rt.L + rt.L / 16 + 1;
    LL = rt.L;
  }
  __shared__ float2 rows[PairShape<L>::ROWS_LDS];
  __shared__ double hist[kMaxBins];
  // per half-space z index: the z part of the phase, 1/W^2 times the mode's
  // weight in the half-space sum (1 on the planes mz = 0 and N/2, which hold
  // their own mirror images, 2 elsewhere), and the LDS row indices of Z(mz)
  // and Z(-mz) (16 bits each)
  __shared__ float4 ztab[MODE != 2 ? kMaxBins + 1 : 1];
  // shell sums: the row pairs that hold a mode inside the last shell,
  // 4 (mx^2 + my^2) < top^2 with top = (2 n_bins + 1) n_dk, column by
  // column (x = 0 .. N/2, in pair_rows' order); colpre[c] is the number of
  // such pairs in the columns before c, coly[c] the largest |my| of column c
  constexpr int kCols = MODE != 2 ? kMaxBins + 2 : 1;
  __shared__ int colpre[kCols];
  __shared__ int coly[kCols];

  const int n = g.n;
  const int mock = blockIdx.y;
  const int ps = threadIdx.x / (2 * TPL);
  const int r = (threadIdx.x / TPL) & 1;
  const int t = threadIdx.x % TPL;
  int64_t npairs = (int64_t)n * n / 2 + 2;
  float2* own_lds = rows + (2 * ps + r) * ROWP;
  const float2* par_lds = rows + (2 * ps + (r ^ 1)) * ROWP;

  if constexpr (MODE != 2) {
    for (int i = threadIdx.x; i < n_bins; i += blockDim.x) hist[i] = 0.0;
    for (int i = threadIdx.x; i <= n / 2; i += blockDim.x) {
      // interlaced: exp(+i pi mz/N); packed: exp(-2 pi i mz/N)
      const float2 ph = IL ? phase[i] : cconj(phase[mod_2n<P2>(2 * i, n)]);
      const float wgt = (i == 0 || i == n / 2) ? 1.0f : 2.0f;
      int ia, ib;
      if constexpr (IL) {
        ia = i;
        ib = neg_mod<P2>(i, n);
      } else {
        // packed rows: N/2 complex values, the plane mz = N/2 folds onto 0
        const int h = n / 2;
        ia = (i == h) ? 0 : i;
        ib = neg_mod<P2>(ia, h);
      }
      const uint32_t zi = (uint32_t)lds_index<1>(ia) | ((uint32_t)lds_index<1>(ib) << 16);
      ztab[i] = make_float4(ph.x, ph.y, wgt * inv_w2[i], __uint_as_float(zi));
    }
    if (threadIdx.x < 64) {
      // wave 0: per-column pair counts and their exclusive scan
      const int h = n / 2, lane = threadIdx.x;
      const int top = (2 * n_bins + 1) * n_dk;
      const int per = (h + 1 + 63) / 64;
      int cnt[(kMaxBins + 1 + 63) / 64];
      int run = 0;
#pragma unroll
      for (int k = 0; k < (kMaxBins + 1 + 63) / 64; ++k) {
        const int c = lane * per + k;
        int ny = 0;
        if (k < per && c <= h) {
          const int lim = top * top - 4 * c * c;  // 4 my^2 < lim
          int ymax = -1;
          if (lim > 0) {
            ymax = (int)sqrtf(0.25f * (float)lim);
            while (ymax >= 0 && 4 * ymax * ymax >= lim) --ymax;
            while (4 * (ymax + 1) * (ymax + 1) < lim) ++ymax;
          }
          coly[c] = ymax;
          if (ymax >= 0) {
            // columns 0 and N/2 hold y = 0 .. N/2 (pair_rows), the others all y
            if (c == 0 || c == h) ny = min(ymax, h) + 1;
            else ny = ymax >= h ? n : 2 * ymax + 1;
          }
        }
        cnt[k] = ny;
        run += ny;
      }
      int incl = run;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      int acc = incl - run;
#pragma unroll
      for (int k = 0; k < (kMaxBins + 1 + 63) / 64; ++k) {
        const int c = lane * per + k;
        if (k < per && c <= h) colpre[c] = acc;
        acc += cnt[k];
      }
      if (lane == 63) colpre[h + 1] = incl;
    }
    __syncthreads();
    npairs = colpre[n / 2 + 1];
  }
  const int64_t ngroups = (npairs + PPB - 1) / PPB;

  for (int64_t pg = blockIdx.x; pg < ngroups; pg += gridDim.x) {
    const int64_t q = pg * PPB + ps;
    const bool valid = q < npairs;
    int xa = 0, ya = 0;
    if (valid) {
      if constexpr (MODE != 2) {
        // the column holding pair q, then its y: 0 .. Y, then N - Y .. N - 1
        const int h = n / 2;
        int lo = 0, hi = h;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (colpre[mid] <= (int)q) lo = mid;
          else hi = mid - 1;
        }
        const int o = (int)q - colpre[lo];
        const int ymax = coly[lo];
        xa = lo;
        ya = (lo == 0 || lo == h || ymax >= h || o <= ymax) ? o : o + n - 2 * ymax - 1;
      } else {
        pair_rows(q, n, xa, ya);
      }
    }
    const int xb = neg_mod<P2>(xa, n), yb = neg_mod<P2>(ya, n);
    const bool self = (xa == xb) && (ya == yb);
    const int xr = r ? xb : xa, yr = r ? yb : ya;
    float2* gp = data + ((int64_t)mock * n + xr) * g.ps + (int64_t)yr * LL;
    float2 v[EPT];
    static_for<0, EPT>([&](auto e) {
      const int j = t + e * TPL;
      v[e] = (valid && (P2 || j < LL)) ? gp[j] : make_float2(0.f, 0.f);
    });
    if constexpr (MODE != 1) {
      if constexpr (P2) line_fft<L, -1, 1>(v, t, own_lds, tw);
      else line_fft_rt<-1, 1>(v, t, own_lds, rt, tw);
    }
    static_for<0, EPT>([&](auto e) {
      const int j = t + e * TPL;
      if (P2 || j < LL) own_lds[lds_index<1>(j)] = v[e];
    });
    __syncthreads();

    const int mxr = signed_freq(xr, n), myr = signed_freq(yr, n);
    if constexpr (MODE != 2) {
      if (valid && !(r == 1 && self)) {
        // this thread's run of half-space z indices; the shell index only
        // grows along it, so it advances by comparing 4|m|^2 with the next
        // shell's lower edge ((2b+1) n_dk)^2 (same rule as shell_of).  The
        // row's modes below the last shell's upper edge, 4 |m|^2 <
        // ((2 n_bins + 1) n_dk)^2, are mz <= zmax; they are split evenly
        // over the row's threads, so no lane idles past the sphere
        const int nm = n / 2 + 1;
        const int r2xy = mxr * mxr + myr * myr;
        const int top = (2 * n_bins + 1) * n_dk;
        const int lim = top * top - 4 * r2xy;  // 4 mz^2 < lim
        int zmax = -1;
        if (lim > 0) {
          zmax = (int)sqrtf(0.25f * (float)lim);
          while (zmax >= 0 && 4 * zmax * zmax >= lim) --zmax;
          while (4 * (zmax + 1) * (zmax + 1) < lim) ++zmax;
          zmax = min(zmax, nm - 1);
        }
        const int per = (zmax + TPL) / TPL;
        const int z0 = t * per;
        const int z1 = min(z0 + per, zmax + 1);
        if (z0 < z1) {
          const float wxy = inv_w2[xr] * inv_w2[yr] * (IL ? 0.0625f : 0.25f);
          const float2 ph_xy = IL ? phase[mod_2n<P2>(mxr + myr, n)] : make_float2(1.0f, 0.0f);
          int m2 = r2xy + z0 * z0;  // |m|^2 of mode mz, advanced by 2 mz + 1 per step
          int b = m2 ? shell_of(m2, n_dk) : 0;
          // the next shell's lower edge ((2b+1) n_dk)^2 and its step to the
          // one after, 8 (b+1) n_dk^2, both advanced by additions
          const int nd2 = n_dk * n_dk;
          int edge = (2 * b + 1) * n_dk;
          edge *= edge;
          int dedge = 8 * (b + 1) * nd2;
          int cur_b = -1;
          float cur = 0.0f;
          for (int mz = z0; mz < z1; m2 += 2 * mz + 1, ++mz) {
            const int m4 = 4 * m2;
            while (edge <= m4) {
              ++b;
              edge += dedge;
              dedge += 8 * nd2;
            }
            // b <= n_bins by the choice of zmax; modes below the first shell
            // (b = 0, the k = 0 mode among them) form a run that is never added
            // the LDS elements of the mode and of its mirror, from the table
            const float4 zt = ztab[mz];
            const uint32_t zi = __float_as_uint(zt.w);
            const float2 za = own_lds[zi & 0xFFFFu];
            const float2 zb = par_lds[zi >> 16];
            const float2 ph = IL ? cmul(ph_xy, make_float2(zt.x, zt.y)) : make_float2(zt.x, zt.y);
            const float val = pair_power(za, zb, ph) * zt.z;
            if (b != cur_b) {
              if (cur_b > 0) atomicAdd(&hist[cur_b - 1], (double)(cur * wxy));
              cur_b = b;
              cur = 0.0f;
            }
            cur += val;
          }
          if (cur_b > 0) atomicAdd(&hist[cur_b - 1], (double)(cur * wxy));
        }
      }
      __syncthreads();
    } else {
      // gradient of the loss with respect to Z at this thread's elements
      const double* cf = coef + (int64_t)mock * n_bins;
      const int xp = r ? xa : xb, yp = r ? ya : yb;  // partner row
      const int mxp = signed_freq(xp, n), myp = signed_freq(yp, n);
      float2 out[EPT];
      static_for<0, EPT>([&](auto e) {
        const int j = t + e * TPL;
        float2 acc = make_float2(0.f, 0.f);
        if (valid) {
          if constexpr (IL) {
            const float2 z1 = (P2 || j < LL) ? own_lds[lds_index<1>(j)] : make_float2(0.f, 0.f);
            const float2 z2 = (P2 || j < LL) ? par_lds[lds_index<1>(neg_mod<P2>(j, n))] : make_float2(0.f, 0.f);
            // (a) mode (own row, j) holds Z(m) = z1
            if (j <= n / 2) {
              const int m2 = mxr * mxr + myr * myr + j * j;
              const int b = m2 ? shell_of(m2, n_dk) : 0;
              if (b >= 1 && b <= n_bins) {
                const float2 c = combined_mode<true, P2>(z1, z2, mxr, myr, j, phase, n);
                const float wgt = (j == 0 || j == n / 2) ? 1.0f : 2.0f;
                const float s = wgt * (float)cf[b - 1] * inv_w2[xr] * inv_w2[yr] * inv_w2[j];
                const float2 gc = cscale(c, s);
                const float2 ph = cconj(phase[mod_2n<P2>(mxr + myr + j, n)]);
                const float2 gf1 = cscale(gc, 0.5f);
                const float2 gf2 = cscale(cmul(ph, gc), 0.5f);
                // dZ(m): 1/2 gF1 + (i/2) gF2
                acc = cadd(acc, make_float2(0.5f * (gf1.x - gf2.y), 0.5f * (gf1.y + gf2.x)));
              }
            }
            // (b) mode (partner row, -j) holds Z(-m') = z1
            const int jp = neg_mod<P2>(j, n);
            if ((P2 || j < LL) && jp <= n / 2) {
              const int m2 = mxp * mxp + myp * myp + jp * jp;
              const int b = m2 ? shell_of(m2, n_dk) : 0;
              if (b >= 1 && b <= n_bins) {
                const float2 c = combined_mode<true, P2>(z2, z1, mxp, myp, jp, phase, n);
                const float wgt = (jp == 0 || jp == n / 2) ? 1.0f : 2.0f;
                const float s = wgt * (float)cf[b - 1] * inv_w2[xp] * inv_w2[yp] * inv_w2[jp];
                const float2 gc = cscale(c, s);
                const float2 ph = cconj(phase[mod_2n<P2>(mxp + myp + jp, n)]);
                const float2 gf1 = cscale(gc, 0.5f);
                const float2 gf2 = cscale(cmul(ph, gc), 0.5f);
                // dZ(-m'): 1/2 conj(gF1) + (i/2) conj(gF2)
                acc = cadd(acc, make_float2(0.5f * (gf1.x + gf2.y), 0.5f * (-gf1.y + gf2.x)));
              }
            }
          } else {
            const int h = n / 2;
            const bool inl = P2 || j < LL;
            const float2 z1 = inl ? own_lds[lds_index<1>(j)] : make_float2(0.f, 0.f);
            const float2 z2 = inl ? par_lds[lds_index<1>(neg_mod<P2>(j, h))] : make_float2(0.f, 0.f);
            // direct sources: modes (own row, mz) with mz = j (and mz = h when j = 0)
            for (int k = 0; k < (!inl ? 0 : (j == 0) ? 2 : 1); ++k) {
              const int mz = k ? h : j;
              const int m2 = mxr * mxr + myr * myr + mz * mz;
              const int b = m2 ? shell_of(m2, n_dk) : 0;
              if (b >= 1 && b <= n_bins) {
                const float2 c = combined_mode<false, P2>(z1, z2, mxr, myr, mz, phase, n);
                const float wgt = (mz == 0 || mz == h) ? 1.0f : 2.0f;
                const float s = wgt * (float)cf[b - 1] * inv_w2[xr] * inv_w2[yr] * inv_w2[mz];
                const float2 gf = cscale(c, s);
                const float2 ph = phase[mod_2n<P2>(2 * mz, n)];  // (cos, sin) of 2 pi mz/N
                // conj(a) = ((1 - sin), cos) / 2
                const float2 ca = make_float2(0.5f * (1.0f - ph.y), 0.5f * ph.x);
                acc = cadd(acc, cmul(ca, gf));
              }
            }
            // conjugate sources: modes (partner row, mz') with -mz' = j mod h (and h when j = 0)
            for (int k = 0; k < (!inl ? 0 : (j == 0) ? 2 : 1); ++k) {
              const int mz = k ? h : neg_mod<P2>(j, h);
              const int m2 = mxp * mxp + myp * myp + mz * mz;
              const int b = m2 ? shell_of(m2, n_dk) : 0;
              if (b >= 1 && b <= n_bins) {
                const float2 c = combined_mode<false, P2>(z2, z1, mxp, myp, mz, phase, n);
                const float wgt = (mz == 0 || mz == h) ? 1.0f : 2.0f;
                const float s = wgt * (float)cf[b - 1] * inv_w2[xp] * inv_w2[yp] * inv_w2[mz];
                const float2 gf = cscale(c, s);
                const float2 ph = phase[mod_2n<P2>(2 * mz, n)];
                // b = ((1 + sin), cos) / 2
                const float2 bb = make_float2(0.5f * (1.0f + ph.y), 0.5f * ph.x);
                acc = cadd(acc, cmul(bb, cconj(gf)));
              }
            }
          }
        }
        out[e] = acc;
      });
      __syncthreads();
      if constexpr (P2) line_fft<L, +1, 1>(out, t, own_lds, tw);
      else line_fft_rt<+1, 1>(out, t, own_lds, rt, tw);
      if (valid && !(r == 1 && self))
        static_for<0, EPT>([&](auto e) {
          const int j = t + e * TPL;
          if (P2 || j < LL) gp[j] = out[e];
        });
      __syncthreads();
    }
  }

  if constexpr (MODE != 2) {
    __syncthreads();
    double* dst = partials + ((int64_t)mock * gridDim.x + blockIdx.x) * n_bins;
    for (int i = threadIdx.x; i < n_bins; i += blockDim.x) dst[i] = hist[i];
  }
}

// P_b = V S_b / (W^2 N_b) [- V sum w^2 / W^2], k_b = k_f K_b / N_b, with W the
// total mass (W = sum w^2 = N_P for equal masses); one wave per
// (bin, set) sums the per-workgroup partials in a fixed order.
__global__ __launch_bounds__(64) void k_power_finalize(const double* __restrict__ partials, int nblk,
                                                       int n_bins, const int64_t* __restrict__ mode_n,
                                                       const double* __restrict__ mode_k,
                                                       const double* __restrict__ norm, double box,
                                                       int subtract, double* k, double* p,
                                                       int64_t* nmodes) {
  const int b = blockIdx.x;
  const int mock = blockIdx.y;
  const double* src = partials + (int64_t)mock * nblk * n_bins + b;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 64) s += src[(int64_t)i * n_bins];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x != 0) return;
  const double vol = box * box * box;
  const double nb = (double)mode_n[b];
  // total mass W (N_P for equal masses); shot noise V (sum w^2 / W) / W
  const double npart = norm[2 * mock];
  double pk = vol * s / (npart * npart * nb);
  if (subtract) pk -= vol * (norm[2 * mock + 1] / npart) / npart;
  if (!(npart > 0.0)) pk = __builtin_nan("");
  const int64_t o = (int64_t)mock * n_bins + b;
  p[o] = pk;
  k[o] = (2.0 * M_PI / box) * mode_k[b] / nb;
  nmodes[o] = mode_n[b];
}

// coefficient 2 g_b V / (N_b N_P^2) of the adjoint spectrum
__global__ void k_adjoint_coef(const double* __restrict__ dldp, int n_bins, const int64_t* __restrict__ mode_n,
                               const double* __restrict__ norm, double box, double* coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int mock = blockIdx.y;
  if (b >= n_bins) return;
  const double vol = box * box * box;
  const double npart = norm[2 * mock];
  const int64_t o = (int64_t)mock * n_bins + b;
  coef[o] = (npart > 0.0) ? 2.0 * dldp[o] * vol / ((double)mode_n[b] * npart * npart) : 0.0;
}

template <int L, bool IL, int MODE>
static hipError_t pairs_t(const Geom& g, const Buffers& b, int nblk, int n_dk, int n_bins,
                          const float2* tw, hipStream_t s) {
  RtLine rt{};
  int threads = 0;
  if constexpr (L == 0) {
    if (!make_rt_line(g.nz, &rt)) return hipErrorInvalidValue;
    threads = 2 * rt_pairs_per_block(rt.tpl) * rt.tpl;
  } else {
    threads = PairShape<L>::THREADS;
  }
  hipLaunchKernelGGL((k_pairs<L, IL, MODE>), dim3(nblk, g.batch), dim3(threads), 0, s,
                     b.grid, g, tw, b.phase, b.inv_w2, n_dk, n_bins, b.partials, b.coef, rt);
  return hipGetLastError();
}

template <int MODE>
static hipError_t pairs_dispatch(const Geom& g, const Buffers& b, int nblk, int n_dk, int n_bins,
                                 hipStream_t s) {
  const float2* tw = b.tw_nz;
#define FSEST_PAIRS_CASE(LL)                                                     \
  case LL:                                                                       \
    return g.il ? pairs_t<LL, true, MODE>(g, b, nblk, n_dk, n_bins, tw, s)       \
                : pairs_t<LL, false, MODE>(g, b, nblk, n_dk, n_bins, tw, s);
  switch ((g.nz & (g.nz - 1)) == 0 ? g.nz : 0) {
    FSEST_PAIRS_CASE(4)
    FSEST_PAIRS_CASE(8)
    FSEST_PAIRS_CASE(16)
    FSEST_PAIRS_CASE(32)
    FSEST_PAIRS_CASE(64)
    FSEST_PAIRS_CASE(128)
    FSEST_PAIRS_CASE(256)
    FSEST_PAIRS_CASE(512)
    FSEST_PAIRS_CASE(1024)
    FSEST_PAIRS_CASE(0)
  }
#undef FSEST_PAIRS_CASE
  return hipErrorInvalidValue;
}

static int pair_blocks(const Geom& g, const Tune& tu) {
  // interlaced rows hold N complex values, packed rows N/2
  int64_t npairs = (int64_t)g.n * g.n / 2 + 2;
  int ppb;
  switch (g.nz) {
    case 4: ppb = PairShape<4>::PPB; break;
    case 8: ppb = PairShape<8>::PPB; break;
    case 16: ppb = PairShape<16>::PPB; break;
    case 32: ppb = PairShape<32>::PPB; break;
    case 64: ppb = PairShape<64>::PPB; break;
    case 128: ppb = PairShape<128>::PPB; break;
    case 256: ppb = PairShape<256>::PPB; break;
    case 512: ppb = PairShape<512>::PPB; break;
    case 1024: ppb = PairShape<1024>::PPB; break;
    default: ppb = rt_pairs_per_block((g.nz + 15) / 16); break;
  }
  int64_t groups = (npairs + ppb - 1) / ppb;
  int64_t nblk = tu.bin_blocks;
  if (nblk > groups) nblk = groups;
  if (nblk > kMaxBinBlocks) nblk = kMaxBinBlocks;
  if (nblk < 1) nblk = 1;
  return (int)nblk;
}

// Shell sums of w |C(m)|^2 / W(m)^2 over the half space for more than two
// grids.  A workgroup takes row pairs (x, y), (-x, -y) as the fused pair
// kernel does and stages both rows of every slab in LDS: with FFT, TPL
// threads per row load it after the x and y passes and run its z transform
// (compile-time length L, or L = 0 for a run-time plan); without, the stored
// spectra are loaded cooperatively.  Then half the threads finish the
// half-space modes of each row (runs of m_z per thread, shells advancing
// along the run).
constexpr int kMultiBlocks = 1024;
constexpr int kMultiThreads = 256;

template <int L, bool FFT>
__global__ __launch_bounds__(1024) void k_multi_pairs(
    float2* __restrict__ data, Geom g, const float2* __restrict__ tw,
    const float2* __restrict__ phase, const float* __restrict__ inv_w2, int n_dk, int n_bins,
    double* __restrict__ partials, RtLine rt) {
  extern __shared__ float2 rows[];  // 2 npair rows of N + N/16 + 1 elements
  __shared__ double hist[kMaxBins];
  constexpr bool P2 = L != 0;
  constexpr int EPT = P2 ? LinePlan<(P2 ? L : 16)>::EPT : 16;
  const int TPL = P2 ? LinePlan<(P2 ? L : 16)>::TPL : rt.tpl;
  const int n = g.n, nm = n / 2 + 1;
  const int mock = blockIdx.y;
  const int rowp = n + n / 16 + 1;
  const int nr = 2 * g.npair;
  const int64_t npairs = (int64_t)n * n / 2 + 2;
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x) hist[i] = 0.0;
  const int half = blockDim.x / 2;
  const int side = threadIdx.x / half;
  const int t = threadIdx.x % half;
  const int per = (nm + half - 1) / half;
  const float inv_g = 1.0f / (float)g.ng;
  const int top = (2 * n_bins + 1) * n_dk;
  for (int64_t pg = blockIdx.x; pg < npairs; pg += gridDim.x) {
    int xa, ya;
    pair_rows(pg, n, xa, ya);
    // a pair whose rows hold no mode inside the last shell, 4 |m|^2 >=
    // ((2 n_bins + 1) n_dk)^2 at mz = 0, adds nothing: skipped by the whole
    // workgroup
    const int mxa = signed_freq(xa, n), mya = signed_freq(ya, n);
    if (4 * (mxa * mxa + mya * mya) >= top * top) continue;
    const int xb = neg_mod<false>(xa, n), yb = neg_mod<false>(ya, n);
    const bool self = (xa == xb) && (ya == yb);
    __syncthreads();  // the previous pair's rows are consumed
    // row r: slab r / 2, side r % 2 (0: (xa, ya), 1: (xb, yb))
    if constexpr (FFT) {
      const int r = threadIdx.x / TPL, tr = threadIdx.x % TPL;
      const int xr = (r & 1) ? xb : xa, yr = (r & 1) ? yb : ya;
      const float2* gp = data + complex_index(g, mock * g.npair + r / 2, xr, yr, 0);
      float2* own = rows + r * rowp;
      float2 v[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int j = tr + e * TPL;
        v[e] = (P2 || j < n) ? gp[j] : make_float2(0.f, 0.f);
      }
      if constexpr (P2) line_fft<(P2 ? L : 16), -1, 1>(v, tr, own, tw);
      else line_fft_rt<-1, 1>(v, tr, own, rt, tw);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int j = tr + e * TPL;
        if (P2 || j < n) own[lds_index<1>(j)] = v[e];
      }
    } else {
      for (int idx = threadIdx.x; idx < nr * n; idx += blockDim.x) {
        const int r = idx / n, j = idx % n;
        const int xr = (r & 1) ? xb : xa, yr = (r & 1) ? yb : ya;
        rows[r * rowp + lds_index<1>(j)] = data[complex_index(g, mock * g.npair + r / 2, xr, yr, j)];
      }
    }
    __syncthreads();
    if (side == 1 && self) continue;
    const int xr = side ? xb : xa, yr = side ? yb : ya;
    const int mx = signed_freq(xr, n), my = signed_freq(yr, n);
    const int z0 = t * per, z1 = min(z0 + per, nm);
    if (z0 >= z1) continue;
    const float wxy = inv_w2[xr] * inv_w2[yr];
    const int r2 = mx * mx + my * my;
    const int m2_0 = r2 + z0 * z0;
    int b = m2_0 ? shell_of(m2_0, n_dk) : 0;
    int edge = (2 * b + 1) * n_dk;
    edge *= edge;
    int cur_b = -1;
    float cur = 0.0f;
    for (int mz = z0; mz < z1; ++mz) {
      const int m4 = 4 * (r2 + mz * mz);
      while (edge <= m4) {
        ++b;
        edge = (2 * b + 1) * n_dk;
        edge *= edge;
      }
      if (b > n_bins) break;
      if (b < 1) continue;  // below the first shell (and the k = 0 mode)
      const int m[3] = {mx, my, mz};
      const int zm = neg_mod<false>(mz, n);
      float2 c = make_float2(0.f, 0.f);
      for (int q = 0; q < g.npair; ++q) {
        const float2 za = rows[(2 * q + side) * rowp + lds_index<1>(mz)];
        const float2 zb = rows[(2 * q + (side ^ 1)) * rowp + lds_index<1>(zm)];
        const float2 f[2] = {make_float2(0.5f * (za.x + zb.x), 0.5f * (za.y - zb.y)),
                             make_float2(0.5f * (za.y + zb.y), 0.5f * (zb.x - za.x))};
        for (int h = 0; h < 2; ++h) {
          const int mk = grid_mask(g.code, 2 * q + h);
          int sj = 0;
          for (int a = 0; a < 3; ++a) sj += ((mk >> a) & 1) ? m[a] : 0;
          c = cadd(c, cmul(phase[mod_2n<false>(sj, n)], f[h]));
        }
      }
      c = cscale(c, inv_g);
      const float wgt = (mz == 0 || mz == n / 2) ? 1.0f : 2.0f;
      const float val = wgt * (c.x * c.x + c.y * c.y) * inv_w2[mz];
      if (b != cur_b) {
        if (cur_b > 0) atomicAdd(&hist[cur_b - 1], (double)(cur * wxy));
        cur_b = b;
        cur = 0.0f;
      }
      cur += val;
    }
    if (cur_b > 0) atomicAdd(&hist[cur_b - 1], (double)(cur * wxy));
  }
  __syncthreads();
  double* dst = partials + ((int64_t)mock * gridDim.x + blockIdx.x) * n_bins;
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x) dst[i] = hist[i];
}

template <int L, bool FFT>
static hipError_t multi_pairs_t(const Geom& g, const Buffers& b, int n_dk, int n_bins,
                                hipStream_t s) {
  RtLine rt{};
  int threads = kMultiThreads;
  if constexpr (FFT) {
    int tpl;
    if constexpr (L == 0) {
      if (!make_rt_line(g.nz, &rt)) return hipErrorInvalidValue;
      tpl = rt.tpl;
    } else {
      tpl = LinePlan<L>::TPL;
    }
    threads = 2 * g.npair * tpl;  // one row of TPL threads per staged row
  }
  const size_t lds = sizeof(float2) * 2 * g.npair * (size_t)(g.n + g.n / 16 + 1);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_multi_pairs<L, FFT>,
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)(sizeof(float2) * 2 * 4 * (1024 + 64 + 1)));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_multi_pairs<L, FFT>), dim3(kMultiBlocks, g.batch), dim3(threads), lds, s,
                     b.grid, g, b.tw_nz, b.phase, b.inv_w2, n_dk, n_bins, b.partials, rt);
  return hipGetLastError();
}

static hipError_t multi_pairs_dispatch(const Geom& g, const Buffers& b, bool do_fft, int n_dk,
                                       int n_bins, hipStream_t s) {
  if (!do_fft) return multi_pairs_t<0, false>(g, b, n_dk, n_bins, s);
  switch ((g.nz & (g.nz - 1)) == 0 ? g.nz : 0) {
    case 8: return multi_pairs_t<8, true>(g, b, n_dk, n_bins, s);
    case 16: return multi_pairs_t<16, true>(g, b, n_dk, n_bins, s);
    case 32: return multi_pairs_t<32, true>(g, b, n_dk, n_bins, s);
    case 64: return multi_pairs_t<64, true>(g, b, n_dk, n_bins, s);
    case 128: return multi_pairs_t<128, true>(g, b, n_dk, n_bins, s);
    case 256: return multi_pairs_t<256, true>(g, b, n_dk, n_bins, s);
    case 512: return multi_pairs_t<512, true>(g, b, n_dk, n_bins, s);
    case 1024: return multi_pairs_t<1024, true>(g, b, n_dk, n_bins, s);
    default: return multi_pairs_t<0, true>(g, b, n_dk, n_bins, s);
  }
}

hipError_t launch_power(const Geom& g, const Buffers& b, const Tune& tu, bool do_fft, int n_dk,
                        int n_bins, int subtract_shot, double* k, double* p, int64_t* nmodes,
                        hipStream_t s) {
  if (g.npair > 1) {
    hipError_t e = multi_pairs_dispatch(g, b, do_fft, n_dk, n_bins, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_power_finalize, dim3(n_bins, g.batch), dim3(64), 0, s, b.partials,
                       kMultiBlocks, n_bins, b.mode_n, b.mode_k, b.norm, g.box, subtract_shot, k, p,
                       nmodes);
    return hipGetLastError();
  }
  const int nblk = pair_blocks(g, tu);
  hipError_t e = do_fft ? pairs_dispatch<0>(g, b, nblk, n_dk, n_bins, s)
                        : pairs_dispatch<1>(g, b, nblk, n_dk, n_bins, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_power_finalize, dim3(n_bins, g.batch), dim3(64), 0, s,
                     b.partials, nblk, n_bins, b.mode_n, b.mode_k, b.norm, g.box, subtract_shot, k, p,
                     nmodes);
  return hipGetLastError();
}

// ---- adjoint with more than two grids (from the stored spectra, after the z
// pass).  (1) C(m) of every half-space mode goes to cbuf; (2) every element
// k of every slab q gets dZ_q(k) from the modes m = k and m' = -k that are
// stored (the transposes of the unpacking, as in the fused pair kernel),
// with dC/dF_j = exp(+i pi s_j/N)/G; (3) the inverse FFT passes follow.
__global__ __launch_bounds__(256) void k_multi_cbuf(const float2* __restrict__ data, Geom g,
                                                    const float2* __restrict__ phase,
                                                    float2* __restrict__ cbuf) {
  const int n = g.n, nh = n / 2 + 1;
  const int64_t per = (int64_t)n * n * nh;
  const int mock = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int mz = (int)(i % nh);
    const int y = (int)((i / nh) % n), x = (int)(i / ((int64_t)n * nh));
    cbuf[(int64_t)mock * per + i] = multi_mode(data, g, mock, signed_freq(x, n), signed_freq(y, n), mz, phase);
  }
}

// gradient with respect to C at half-space mode (x, y, mz) times the half-space weight and
// 1/W^2 (zero outside the bins)
__device__ __forceinline__ float2 multi_grad_c(const float2* __restrict__ cb, const Geom& g, int x,
                                               int y, int mz, const double* __restrict__ cf,
                                               const float* __restrict__ inv_w2, int n_dk,
                                               int n_bins) {
  const int n = g.n, nh = n / 2 + 1;
  const int mx = signed_freq(x, n), my = signed_freq(y, n);
  const int m2 = mx * mx + my * my + mz * mz;
  const int b = m2 ? shell_of(m2, n_dk) : 0;
  if (b < 1 || b > n_bins) return make_float2(0.f, 0.f);
  const float wgt = (mz == 0 || mz == n / 2) ? 1.0f : 2.0f;
  const float s = wgt * (float)cf[b - 1] * inv_w2[x] * inv_w2[y] * inv_w2[mz];
  return cscale(cb[((int64_t)x * n + y) * nh + mz], s);
}

__global__ __launch_bounds__(256) void k_multi_adjoint(float2* __restrict__ data, Geom g,
                                                       const float2* __restrict__ cbuf,
                                                       const float2* __restrict__ phase,
                                                       const float* __restrict__ inv_w2,
                                                       const double* __restrict__ coef, int n_dk,
                                                       int n_bins) {
  const int n = g.n, nh = n / 2 + 1;
  const int64_t n3 = (int64_t)n * n * n;
  const int slab = blockIdx.y;
  const int mock = slab / g.npair, q = slab % g.npair;
  const float2* cb = cbuf + (int64_t)mock * n * n * nh;
  const double* cf = coef + (int64_t)mock * n_bins;
  const float inv_g = 1.0f / (float)g.ng;
  const int ma = grid_mask(g.code, 2 * q), mb = grid_mask(g.code, 2 * q + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(i % n), y = (int)((i / n) % n), x = (int)(i / ((int64_t)n * n));
    float2 acc = make_float2(0.f, 0.f);
    // (a) m = k stored: Z_q(k) enters F_2q(m) and F_2q+1(m) directly
    if (z <= n / 2) {
      const float2 gc = multi_grad_c(cb, g, x, y, z, cf, inv_w2, n_dk, n_bins);
      const int m[3] = {signed_freq(x, n), signed_freq(y, n), z};
      int sa = 0, sb = 0;
      for (int a = 0; a < 3; ++a) {
        sa += ((ma >> a) & 1) ? m[a] : 0;
        sb += ((mb >> a) & 1) ? m[a] : 0;
      }
      const float2 ga = cscale(cmul(cconj(phase[mod_2n<false>(sa, n)]), gc), inv_g);
      const float2 gb = cscale(cmul(cconj(phase[mod_2n<false>(sb, n)]), gc), inv_g);
      acc = cadd(acc, make_float2(0.5f * (ga.x - gb.y), 0.5f * (ga.y + gb.x)));
    }
    // (b) m' = -k stored: Z_q(k) = Z_q(-m') enters through the conjugate
    const int xp = neg_mod<false>(x, n), yp = neg_mod<false>(y, n), zp = neg_mod<false>(z, n);
    if (zp <= n / 2) {
      const float2 gc = multi_grad_c(cb, g, xp, yp, zp, cf, inv_w2, n_dk, n_bins);
      const int m[3] = {signed_freq(xp, n), signed_freq(yp, n), zp};
      int sa = 0, sb = 0;
      for (int a = 0; a < 3; ++a) {
        sa += ((ma >> a) & 1) ? m[a] : 0;
        sb += ((mb >> a) & 1) ? m[a] : 0;
      }
      const float2 ga = cscale(cmul(cconj(phase[mod_2n<false>(sa, n)]), gc), inv_g);
      const float2 gb = cscale(cmul(cconj(phase[mod_2n<false>(sb, n)]), gc), inv_g);
      acc = cadd(acc, make_float2(0.5f * (ga.x + gb.y), 0.5f * (-ga.y + gb.x)));
    }
    data[complex_index(g, slab, x, y, z)] = acc;
  }
}

hipError_t launch_multi_adjoint(const Geom& g, const Buffers& b, const double* dldp, int n_dk,
                                int n_bins, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_coef, dim3((n_bins + 127) / 128, g.batch), dim3(128), 0, s, dldp,
                     n_bins, b.mode_n, b.norm, g.box, b.coef);
  hipLaunchKernelGGL(k_multi_cbuf, dim3(4096, g.batch), dim3(256), 0, s, b.grid, g, b.phase, b.cbuf);
  hipLaunchKernelGGL(k_multi_adjoint, dim3(4096, g.batch * g.npair), dim3(256), 0, s, b.grid, g,
                     b.cbuf, b.phase, b.inv_w2, b.coef, n_dk, n_bins);
  return hipGetLastError();
}

hipError_t launch_adjoint_spectrum(const Geom& g, const Buffers& b, const Tune& tu,
                                   const double* dldp, int n_dk, int n_bins, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_coef, dim3((n_bins + 127) / 128, g.batch), dim3(128), 0, s, dldp,
                     n_bins, b.mode_n, b.norm, g.box, b.coef);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nblk = pair_blocks(g, tu);
  return pairs_dispatch<2>(g, b, nblk, n_dk, n_bins, s);
}

// ------------------------------------------------------------------ mode table
__global__ __launch_bounds__(256) void k_mode_table(Geom g, int n_dk, int n_bins,
                                                    uint64_t* __restrict__ pn, double* __restrict__ pk) {
  __shared__ unsigned long long hn[kMaxBins];
  __shared__ double hk[kMaxBins];
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x) { hn[i] = 0ull; hk[i] = 0.0; }
  __syncthreads();
  const int n = g.n, nm = n / 2 + 1;
  constexpr int CH = 16;
  const int chunks = (nm + CH - 1) / CH;
  const int64_t items = (int64_t)n * n * chunks;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = it / chunks;
    const int ch = (int)(it % chunks);
    const int mx = signed_freq((int)(row / n), n), my = signed_freq((int)(row % n), n);
    const int r2 = mx * mx + my * my;
    int cur_b = -1;
    unsigned long long cn = 0;
    double ck = 0.0;
    for (int mz = ch * CH; mz < min(ch * CH + CH, nm); ++mz) {
      const int m2 = r2 + mz * mz;
      if (m2 == 0) continue;
      const int b = shell_of(m2, n_dk);
      if (b < 1 || b > n_bins) continue;
      const int w = (mz == 0 || mz == n / 2) ? 1 : 2;
      if (b != cur_b) {
        if (cur_b > 0) { atomicAdd(&hn[cur_b - 1], cn); atomicAdd(&hk[cur_b - 1], ck); }
        cur_b = b; cn = 0; ck = 0.0;
      }
      cn += w;
      ck += w * sqrt((double)m2);
    }
    if (cur_b > 0) { atomicAdd(&hn[cur_b - 1], cn); atomicAdd(&hk[cur_b - 1], ck); }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x) {
    pn[(int64_t)blockIdx.x * n_bins + i] = hn[i];
    pk[(int64_t)blockIdx.x * n_bins + i] = hk[i];
  }
}

__global__ void k_mode_finalize(const uint64_t* pn, const double* pk, int nblk, int n_bins,
                                int64_t* mode_n, double* mode_k) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  uint64_t c = 0;
  double kk = 0.0;
  for (int i = 0; i < nblk; ++i) {
    c += pn[(int64_t)i * n_bins + b];
    kk += pk[(int64_t)i * n_bins + b];
  }
  mode_n[b] = (int64_t)c;
  mode_k[b] = kk;
}

hipError_t launch_mode_table(const Geom& g, const Buffers& b, int n_dk, int n_bins, hipStream_t s) {
  const int nblk = 512;
  hipLaunchKernelGGL(k_mode_table, dim3(nblk), dim3(256), 0, s, g, n_dk, n_bins,
                     b.mode_partials_n, b.mode_partials_k);
  hipLaunchKernelGGL(k_mode_finalize, dim3((n_bins + 127) / 128), dim3(128), 0, s,
                     b.mode_partials_n, b.mode_partials_k, nblk, n_bins, b.mode_n, b.mode_k);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sampled delta
// delta(m) = C(m) / (N_P W(m)) at signed modes, from the stored full spectrum.
// delta(m) = C(m) / (N_P W(m)) at half-space mode m from the stored
// spectrum Z (after the z pass), in FP64: the estimator's Fourier density
// (eqs. intdelta, windowcorrection), normalised like the direct sum.
__device__ void delta_at(const float2* __restrict__ data, const Geom& g, int mock, int mx, int my,
                         int mz, double npart, double& re, double& im) {
  const int n = g.n;
  const int x = ((mx % n) + n) % n, y = ((my % n) + n) % n;
  const int xm = neg_mod<false>(x, n), ym = neg_mod<false>(y, n);
  const int L = g.nz;
  const int z = ((mz % L) + L) % L, zm = neg_mod<false>(z, L);
  double cr, ci;
  if (g.npair > 1) {
    // more than two grids: (1/G) sum_j F_j exp(+i pi s_j / N)
    const int m[3] = {mx, my, mz};
    cr = ci = 0.0;
    for (int q = 0; q < g.npair; ++q) {
      const float2 za = data[complex_index(g, mock * g.npair + q, x, y, z)];
      const float2 zb = data[complex_index(g, mock * g.npair + q, xm, ym, zm)];
      const double fr[2] = {0.5 * ((double)za.x + zb.x), 0.5 * ((double)za.y + zb.y)};
      const double fi[2] = {0.5 * ((double)za.y - zb.y), 0.5 * ((double)zb.x - za.x)};
      for (int h = 0; h < 2; ++h) {
        const int mk = grid_mask(g.code, 2 * q + h);
        int sj = 0;
        for (int a = 0; a < 3; ++a) sj += ((mk >> a) & 1) ? m[a] : 0;
        double sn, cs;
        sincospi((double)sj / n, &sn, &cs);
        cr += cs * fr[h] - sn * fi[h];
        ci += cs * fi[h] + sn * fr[h];
      }
    }
    cr /= g.ng;
    ci /= g.ng;
    double w = 1.0;
    for (int a = 0; a < 3; ++a) {
      if (m[a] != 0) {
        const double xx = (double)m[a] / n;
        const double sc = sinpi(xx) / (M_PI * xx);
        for (int k = 0; k < g.order; ++k) w *= sc;
      }
    }
    re = cr / (npart * w);
    im = ci / (npart * w);
    return;
  }
  const float2 za = data[complex_index(g, mock, x, y, z)];
  const float2 zb = data[complex_index(g, mock, xm, ym, zm)];
  const double f1r = 0.5 * ((double)za.x + zb.x), f1i = 0.5 * ((double)za.y - zb.y);
  const double f2r = 0.5 * ((double)za.y + zb.y), f2i = 0.5 * ((double)zb.x - za.x);
  if (g.il) {
    double s, c;
    sincospi((double)(mx + my + mz) / n, &s, &c);
    cr = 0.5 * (f1r + c * f2r - s * f2i);
    ci = 0.5 * (f1i + c * f2i + s * f2r);
  } else {
    double s, c;
    sincospi(-2.0 * mz / n, &s, &c);
    cr = f1r + c * f2r - s * f2i;
    ci = f1i + c * f2i + s * f2r;
  }
  double w = 1.0;
  const int mm[3] = {mx, my, mz};
  for (int a = 0; a < 3; ++a) {
    if (mm[a] != 0) {
      const double xx = (double)mm[a] / n;
      const double sc = sinpi(xx) / (M_PI * xx);
      for (int k = 0; k < g.order; ++k) w *= sc;
    }
  }
  const double d = npart * w;
  re = cr / d;
  im = ci / d;
}

__global__ void k_sample_delta(const float2* __restrict__ data, Geom g, int mock,
                               const int32_t* __restrict__ modes, int64_t nm,
                               const double* __restrict__ norm, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nm) return;
  delta_at(data, g, mock, modes[3 * i], modes[3 * i + 1], modes[3 * i + 2], norm[2 * mock],
           out[2 * i], out[2 * i + 1]);
}

// every half-space mode, index (ix * N + iy) * (N/2 + 1) + m_z (FFT indices
// ix, iy; index N/2 is +N/2)
__global__ void k_export_delta(const float2* __restrict__ data, Geom g, int mock,
                               const double* __restrict__ norm, double* __restrict__ out) {
  const int n = g.n, nh = n / 2 + 1;
  const int64_t nm = (int64_t)n * n * nh;
  const double npart = norm[2 * mock];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nm;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int mz = (int)(i % nh);
    const int iy = (int)((i / nh) % n), ix = (int)(i / ((int64_t)n * nh));
    delta_at(data, g, mock, signed_freq(ix, n), signed_freq(iy, n), mz, npart, out[2 * i],
             out[2 * i + 1]);
  }
}

hipError_t launch_export_delta(const Geom& g, const Buffers& b, int mock, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_export_delta, dim3(4096), dim3(256), 0, s, b.grid, g, mock, b.norm, out);
  return hipGetLastError();
}

// Shell sums of w Re(a conj(b)) over the half spectrum (a, b complex128 in
// k_export_delta's order; b == a when b is null), w = 1 on m_z in {0, N/2}
// and 2 elsewhere, shells as shell_of.  Per-workgroup partial histograms,
// then the same fixed-order reduction as the P(k) pass.
constexpr int kSpecBlocks = 512;

__global__ __launch_bounds__(256) void k_spec_bins(const double* __restrict__ a,
                                                   const double* __restrict__ bb, Geom g, int n_dk,
                                                   int n_bins, double* __restrict__ partials) {
  __shared__ double hist[kMaxBins];
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x) hist[i] = 0.0;
  __syncthreads();
  const int n = g.n, nh = n / 2 + 1;
  constexpr int CH = 16;
  const int chunks = (nh + CH - 1) / CH;
  const int64_t items = (int64_t)n * n * chunks;
  const double* b2 = bb ? bb : a;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = it / chunks;
    const int ch = (int)(it % chunks);
    const int mx = signed_freq((int)(row / n), n), my = signed_freq((int)(row % n), n);
    const int r2 = mx * mx + my * my;
    int cur_b = -1;
    double cur = 0.0;
    for (int mz = ch * CH; mz < (ch + 1) * CH && mz < nh; ++mz) {
      const int m2 = r2 + mz * mz;
      if (m2 == 0) continue;
      const int b = shell_of(m2, n_dk);
      if (b < 1 || b > n_bins) continue;
      const int64_t i = row * nh + mz;
      const double v = a[2 * i] * b2[2 * i] + a[2 * i + 1] * b2[2 * i + 1];
      const double w = (mz == 0 || mz == n / 2) ? 1.0 : 2.0;
      if (b != cur_b) {
        if (cur_b > 0) atomicAdd(&hist[cur_b - 1], cur);
        cur_b = b;
        cur = 0.0;
      }
      cur += w * v;
    }
    if (cur_b > 0) atomicAdd(&hist[cur_b - 1], cur);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_bins; i += blockDim.x)
    partials[(int64_t)blockIdx.x * n_bins + i] = hist[i];
}

__global__ __launch_bounds__(64) void k_spec_finalize(const double* __restrict__ partials, int nblk,
                                                      int n_bins,
                                                      const int64_t* __restrict__ mode_n,
                                                      const double* __restrict__ mode_k, double box,
                                                      double shot, double* k, double* p,
                                                      int64_t* nmodes) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 64) s += partials[(int64_t)i * n_bins + b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x != 0) return;
  const double vol = box * box * box;
  const double nb = (double)mode_n[b];
  p[b] = vol * s / nb - shot;
  k[b] = (2.0 * M_PI / box) * mode_k[b] / nb;
  nmodes[b] = mode_n[b];
}

hipError_t launch_spectrum_power(const Geom& g, const Buffers& b, const double* a, const double* bb,
                                 int n_dk, int n_bins, double shot, double* k, double* p,
                                 int64_t* nmodes, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_bins, dim3(kSpecBlocks), dim3(256), 0, s, a, bb, g, n_dk, n_bins,
                     b.partials);
  hipLaunchKernelGGL(k_spec_finalize, dim3(n_bins), dim3(64), 0, s, b.partials, kSpecBlocks,
                     n_bins, b.mode_n, b.mode_k, g.box, shot, k, p, nmodes);
  return hipGetLastError();
}

hipError_t launch_sample_delta(const Geom& g, const Buffers& b, int mock, const int32_t* modes,
                               int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_delta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b.grid, g,
                     mock, modes, n, b.norm, out);
  return hipGetLastError();
}

}  // namespace fsest
