// 3D complex FFT passes over the grid (Sec. 2.3: one forward transform per
// grid; the two real grids travel as one complex grid rho1 + i rho2, or as a
// real grid packed pairwise along z when there is no interlacing).
//
// The grid is [batch][N][N][nz] complex, z contiguous.  One pass per axis:
//   z (contiguous): k_fft_rows, LPB rows per workgroup, padded rows in LDS;
//   x, y (strided): k_fft_cols, C adjacent lines per workgroup so that every
//                   global access is a run of C complex values (C*8 bytes),
//                   lines interleaved in LDS; k_fft_cols_pf, the same with a
//                   fixed grid that prefetches the next chunk, where one
//                   workgroup fills a CU's LDS.
// Every workgroup owns its lines, so the passes run in place.  Lengths with
// factors 3 and 5 take the run-time-planned kernels (k_*_rt).
#include "fft_line.hpp"
#include "fsest_internal.hpp"

namespace fsest {

template <int L>
struct RowShape {
  static constexpr int TPL = LinePlan<L>::TPL;
  static constexpr int LPB = (256 / TPL) > 0 ? (256 / TPL) : 1;
};

template <int L, int DIR>
__global__ __launch_bounds__(RowShape<L>::LPB * RowShape<L>::TPL) void k_fft_rows(
    float2* __restrict__ data, int64_t nrows, int rows_per_plane, int64_t plane_stride,
    const float2* __restrict__ tw) {
  constexpr int TPL = RowShape<L>::TPL;
  constexpr int LPB = RowShape<L>::LPB;
  constexpr int EPT = LinePlan<L>::EPT;
  constexpr int ROWP = LdsLine<L>::padded;
  __shared__ float2 lds[LPB * ROWP];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const int64_t row = (int64_t)blockIdx.x * LPB + line;
  const bool valid = row < nrows;
  float2* p = data + (row / rows_per_plane) * plane_stride + (row % rows_per_plane) * L;
  float2 v[EPT];
  static_for<0, EPT>([&](auto e) { v[e] = valid ? p[t + e * TPL] : make_float2(0.f, 0.f); });
  line_fft<L, DIR, 1>(v, t, lds + line * ROWP, tw);
  if (valid) static_for<0, EPT>([&](auto e) { p[t + e * TPL] = v[e]; });
}

// spread > 0: the chunks of one outer block form spread rows of
// chunks_per_outer / spread chunks, and consecutive workgroups take the same
// chunk of consecutive rows (for the x pass: consecutive y at one z range,
// measured 5.02 -> 4.91 ms at 1024^3 against consecutive z chunks of one y).
template <int L, int DIR, int C>
__global__ __launch_bounds__(C * LinePlan<L>::TPL) void k_fft_cols(
    float2* __restrict__ data, int64_t elem_stride, int64_t chunks_per_outer, int64_t outer_stride,
    const float2* __restrict__ tw, int64_t spread) {
  constexpr int TPL = LinePlan<L>::TPL;
  constexpr int EPT = LinePlan<L>::EPT;
  extern __shared__ float2 lds_dyn[];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t outer = blockIdx.x / chunks_per_outer;
  const int64_t ib = blockIdx.x % chunks_per_outer;
  const int64_t ic = spread ? (ib % spread) * (chunks_per_outer / spread) + ib / spread : ib;
  float2* p = data + outer * outer_stride + ic * C + c;
  float2 v[EPT];
  static_for<0, EPT>([&](auto e) { v[e] = p[(int64_t)(t + e * TPL) * elem_stride]; });
  line_fft<L, DIR, C>(v, t, lds_dyn + c, tw);
  static_for<0, EPT>([&](auto e) { p[(int64_t)(t + e * TPL) * elem_stride] = v[e]; });
}

// The same pass for a workgroup that fills a CU's LDS alone (L C >= 16384):
// a fixed grid of workgroups walks the chunks b = blockIdx.x + k gridDim.x,
// and each loads the next chunk's elements into registers before the
// transform of the current one, so that a CU's loads stay in flight while
// it transforms and stores.  1024-point lines take the 32 x 32 plan (32
// threads per line, one LDS exchange).  At 1024^3 (probe, 16 lines per
// workgroup): x pass 4.91 ms one chunk per workgroup, 4.26 ms prefetching
// with the 16 x 16 x 4 plan, 3.93 ms with the 32 x 32 plan; y pass 4.00,
// 3.96 and 3.65 ms.  Addresses are a uniform chunk base plus a 32-bit
// per-thread byte offset (the host checks that it fits).  The twiddle
// pointer passes through an empty asm statement in every iteration so that
// the compiler reloads the twiddles per chunk instead of keeping them all in
// registers (which spills).
template <int L>
struct PfPlan {
  static constexpr int TPL = L == 1024 ? 32 : LinePlan<L>::TPL;
  static constexpr int EPT = L / TPL;
};

template <int L, int DIR, int C>
__global__ __launch_bounds__(C * PfPlan<L>::TPL) void k_fft_cols_pf(
    float2* __restrict__ data, int64_t elem_stride, int64_t chunks_per_outer, int64_t outer_stride,
    const float2* __restrict__ tw, int64_t spread, int64_t total) {
  constexpr int TPL = PfPlan<L>::TPL;
  constexpr int EPT = PfPlan<L>::EPT;
  extern __shared__ float2 lds_dyn[];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  auto chunk_base = [&](int64_t b) {
    const int64_t outer = b / chunks_per_outer;
    const int64_t ib = b % chunks_per_outer;
    const int64_t ic = spread ? (ib % spread) * (chunks_per_outer / spread) + ib / spread : ib;
    return (char*)(data + outer * outer_stride + ic * C);
  };
  const uint32_t voff = (uint32_t)((c + (int64_t)t * elem_stride) * (int64_t)sizeof(float2));
  const int64_t estep = (int64_t)TPL * elem_stride * (int64_t)sizeof(float2);
  int64_t b = blockIdx.x;
  if (b >= total) return;
  float2 next[EPT];
  {
    const char* q = chunk_base(b);
    static_for<0, EPT>([&](auto e) { next[e] = *(const float2*)(q + e * estep + voff); });
  }
  for (; b < total; b += gridDim.x) {
    float2 v[EPT];
    static_for<0, EPT>([&](auto e) { v[e] = next[e]; });
    char* p = chunk_base(b);
    if (b + gridDim.x < total) {
      const char* q = chunk_base(b + gridDim.x);
      static_for<0, EPT>([&](auto e) { next[e] = *(const float2*)(q + e * estep + voff); });
    }
    const float2* twb = tw;
    asm volatile("" : "+s"(twb));
    if constexpr (L == 1024) line_fft_1024_r32<DIR, C>(v, t, lds_dyn + c, twb);
    else line_fft<L, DIR, C>(v, t, lds_dyn + c, twb);
    static_for<0, EPT>([&](auto e) { *(float2*)(p + e * estep + voff) = v[e]; });
  }
}

template <int L, int DIR>
static hipError_t rows_t(float2* data, int64_t nrows, int rpp, int64_t ps, const float2* tw,
                         hipStream_t s) {
  const unsigned blocks = (unsigned)((nrows + RowShape<L>::LPB - 1) / RowShape<L>::LPB);
  hipLaunchKernelGGL((k_fft_rows<L, DIR>), dim3(blocks), dim3(RowShape<L>::LPB * RowShape<L>::TPL),
                     0, s, data, nrows, rpp, ps, tw);
  return hipGetLastError();
}

template <int L, int DIR, int C>
static hipError_t cols_tc(float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                          int64_t outer_stride, int64_t spread, int cus, const float2* tw,
                          hipStream_t s) {
  const int64_t chunks = inner / C;
  if (spread && chunks % spread != 0) spread = 0;
  const size_t lds = sizeof(float2) * (size_t)L * C;
  if constexpr (L * C >= 16384) {
    const int64_t total = chunks * outer;
    const int64_t span = ((int64_t)(PfPlan<L>::TPL - 1) * elem_stride + C) * (int64_t)sizeof(float2);
    if (cus > 0 && span < ((int64_t)1 << 32)) {
      static bool pf_attr_set = false;
      if (!pf_attr_set) {
        (void)hipFuncSetAttribute((const void*)k_fft_cols_pf<L, DIR, C>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        pf_attr_set = true;
      }
      const int64_t grid = total < 2 * (int64_t)cus ? total : 2 * (int64_t)cus;
      hipLaunchKernelGGL((k_fft_cols_pf<L, DIR, C>), dim3((unsigned)grid),
                         dim3(C * PfPlan<L>::TPL), lds, s, data, elem_stride, chunks,
                         outer_stride, tw, spread, total);
      return hipGetLastError();
    }
  }
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_fft_cols<L, DIR, C>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr_set = true;
  }
  hipLaunchKernelGGL((k_fft_cols<L, DIR, C>), dim3((unsigned)(chunks * outer)),
                     dim3(C * LinePlan<L>::TPL), lds, s, data, elem_stride, chunks, outer_stride, tw,
                     spread);
  return hipGetLastError();
}

template <int L, int DIR>
static hipError_t cols_t(float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                         int64_t outer_stride, int64_t spread, int c, int cus, const float2* tw,
                         hipStream_t s) {
  if (c >= 16 && inner % 16 == 0)
    return cols_tc<L, DIR, 16>(data, elem_stride, inner, outer, outer_stride, spread, cus, tw, s);
  if (c >= 8 && inner % 8 == 0)
    return cols_tc<L, DIR, 8>(data, elem_stride, inner, outer, outer_stride, spread, cus, tw, s);
  return cols_tc<L, DIR, 4>(data, elem_stride, inner, outer, outer_stride, spread, cus, tw, s);
}

// ---- lengths 2^a 3^b 5^c (run-time plan) ----
// rows: lpb = 256 / tpl lines per workgroup, padded rows in LDS (at most
// (256 / tpl) (L + L/16 + 1) <= 4608 elements since L <= 16 tpl)
constexpr int kRtRowsLds = 4608;

template <int DIR>
__global__ __launch_bounds__(256) void k_fft_rows_rt(float2* __restrict__ data, int64_t nrows,
                                                     int rows_per_plane, int64_t plane_stride,
                                                     const float2* __restrict__ tw, RtLine pl) {
  __shared__ float2 lds[kRtRowsLds];
  const int L = pl.L, tpl = pl.tpl;
  const int lpb = 256 / tpl;
  const int rowp = L + L / 16 + 1;
  const int line = threadIdx.x / tpl, t = threadIdx.x % tpl;
  const int64_t row = (int64_t)blockIdx.x * lpb + line;
  const bool valid = row < nrows;
  float2* p = data + (row / rows_per_plane) * plane_stride + (row % rows_per_plane) * L;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int j = t + e * tpl;
    v[e] = (valid && j < L) ? p[j] : make_float2(0.f, 0.f);
  }
  line_fft_rt<DIR, 1>(v, t, lds + line * rowp, pl, tw);
  if (valid) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = t + e * tpl;
      if (j < L) p[j] = v[e];
    }
  }
}

// strided lines: C adjacent lines per workgroup, interleaved in LDS; the
// last chunk of a row may be partial (lines past `inner` load zeros and are
// not stored)
template <int DIR, int C>
__global__ __launch_bounds__(1024) void k_fft_cols_rt(float2* __restrict__ data, int64_t elem_stride,
                                                      int64_t inner, int64_t chunks_per_outer,
                                                      int64_t outer_stride,
                                                      const float2* __restrict__ tw, RtLine pl) {
  extern __shared__ float2 lds_dyn[];
  const int L = pl.L, tpl = pl.tpl;
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t outer = blockIdx.x / chunks_per_outer;
  const int64_t ic = blockIdx.x % chunks_per_outer;
  const bool valid = ic * C + c < inner;
  const float2* p = data + outer * outer_stride + ic * C + c;
  float2 v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int j = t + e * tpl;
    v[e] = (valid && j < L) ? p[(int64_t)j * elem_stride] : make_float2(0.f, 0.f);
  }
  line_fft_rt<DIR, C>(v, t, lds_dyn + c, pl, tw);
  // the store addresses are formed again from a base the compiler cannot
  // match with the loads' (an empty asm statement), so that the 16 64-bit
  // load addresses are not kept live across the transform (they spilled)
  float2* ds = data;
  asm volatile("" : "+s"(ds));
  float2* q = ds + outer * outer_stride + ic * C + c;
  if (valid) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = t + e * tpl;
      if (j < L) q[(int64_t)j * elem_stride] = v[e];
    }
  }
}

template <int DIR>
static hipError_t rows_rt(int L, float2* data, int64_t nrows, int rpp, int64_t ps, const float2* tw,
                          hipStream_t s) {
  RtLine pl;
  if (!make_rt_line(L, &pl)) return hipErrorInvalidValue;
  const int lpb = 256 / pl.tpl;
  const unsigned blocks = (unsigned)((nrows + lpb - 1) / lpb);
  hipLaunchKernelGGL((k_fft_rows_rt<DIR>), dim3(blocks), dim3(lpb * pl.tpl), 0, s, data, nrows, rpp,
                     ps, tw, pl);
  return hipGetLastError();
}

template <int DIR>
static hipError_t cols_rt(int L, float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                          int64_t outer_stride, const float2* tw, hipStream_t s) {
  constexpr int C = 16;  // 16 * tpl <= 1024 threads and 16 L <= 16384 elements of LDS
  RtLine pl;
  if (!make_rt_line(L, &pl) || C * pl.tpl > 1024) return hipErrorInvalidValue;
  const int64_t chunks = (inner + C - 1) / C;
  const size_t lds = sizeof(float2) * (size_t)L * C;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_fft_cols_rt<DIR, C>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(float2) * 1024 * C));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_fft_cols_rt<DIR, C>), dim3((unsigned)(chunks * outer)), dim3(C * pl.tpl),
                     lds, s, data, elem_stride, inner, chunks, outer_stride, tw, pl);
  return hipGetLastError();
}

template <int DIR>
static hipError_t rows_dir(int L, float2* data, int64_t nrows, int rpp, int64_t ps,
                           const float2* tw, hipStream_t s) {
  switch (L) {
    case 4: return rows_t<4, DIR>(data, nrows, rpp, ps, tw, s);
    case 8: return rows_t<8, DIR>(data, nrows, rpp, ps, tw, s);
    case 16: return rows_t<16, DIR>(data, nrows, rpp, ps, tw, s);
    case 32: return rows_t<32, DIR>(data, nrows, rpp, ps, tw, s);
    case 64: return rows_t<64, DIR>(data, nrows, rpp, ps, tw, s);
    case 128: return rows_t<128, DIR>(data, nrows, rpp, ps, tw, s);
    case 256: return rows_t<256, DIR>(data, nrows, rpp, ps, tw, s);
    case 512: return rows_t<512, DIR>(data, nrows, rpp, ps, tw, s);
    case 1024: return rows_t<1024, DIR>(data, nrows, rpp, ps, tw, s);
    default: return rows_rt<DIR>(L, data, nrows, rpp, ps, tw, s);
  }
}

template <int DIR>
static hipError_t cols_dir(int L, float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                           int64_t outer_stride, int64_t spread, int c, int cus, const float2* tw,
                           hipStream_t s) {
#define FSEST_COLS_CASE(LL) \
  case LL: \
    return cols_t<LL, DIR>(data, elem_stride, inner, outer, outer_stride, spread, c, cus, tw, s);
  switch (L) {
    FSEST_COLS_CASE(8)
    FSEST_COLS_CASE(16)
    FSEST_COLS_CASE(32)
    FSEST_COLS_CASE(64)
    FSEST_COLS_CASE(128)
    FSEST_COLS_CASE(256)
    FSEST_COLS_CASE(512)
    FSEST_COLS_CASE(1024)
    default: return cols_rt<DIR>(L, data, elem_stride, inner, outer, outer_stride, tw, s);
  }
#undef FSEST_COLS_CASE
}

hipError_t launch_fft_rows_len(int L, float2* data, int64_t nrows, int rows_per_plane,
                               int64_t plane_stride, int dir, const float2* tw, hipStream_t s) {
  return dir < 0 ? rows_dir<-1>(L, data, nrows, rows_per_plane, plane_stride, tw, s)
                 : rows_dir<+1>(L, data, nrows, rows_per_plane, plane_stride, tw, s);
}

hipError_t launch_fft_cols_len(int L, float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                               int64_t outer_stride, int dir, int c, const float2* tw, hipStream_t s) {
  return dir < 0 ? cols_dir<-1>(L, data, elem_stride, inner, outer, outer_stride, 0, c, 0, tw, s)
                 : cols_dir<+1>(L, data, elem_stride, inner, outer, outer_stride, 0, c, 0, tw, s);
}

hipError_t launch_fft_axis(const Geom& g, float2* data, int axis, int dir, int batch, int nz_len,
                           const float2* tw_axis, const Tune& tu, hipStream_t s) {
  const int64_t n = g.n, nz = nz_len, ps = g.ps;
  if (axis == 2) {
    const int64_t nrows = (int64_t)batch * n * n;
    return dir < 0 ? rows_dir<-1>((int)nz, data, nrows, (int)n, ps, tw_axis, s)
                   : rows_dir<+1>((int)nz, data, nrows, (int)n, ps, tw_axis, s);
  }
  int64_t elem_stride, inner, outer, outer_stride, spread;
  if (axis == 0) {
    // x lines at each (y, z): workgroups spread over y first
    elem_stride = ps;
    inner = n * nz;
    outer = batch;
    outer_stride = n * ps;
    spread = n;
  } else {
    elem_stride = nz;
    inner = nz;
    outer = (int64_t)batch * n;
    outer_stride = ps;
    spread = 0;
  }
  return dir < 0 ? cols_dir<-1>((int)n, data, elem_stride, inner, outer, outer_stride, spread,
                                tu.cols_c, tu.cus, tw_axis, s)
                 : cols_dir<+1>((int)n, data, elem_stride, inner, outer, outer_stride, spread,
                                tu.cols_c, tu.cus, tw_axis, s);
}

}  // namespace fsest
