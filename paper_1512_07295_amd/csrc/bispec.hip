// FFT-shell bispectrum (Sec. 4.1, eqs. Best, VBest, Best2, IntI).
//
// For shells b of width n_dk k_f the estimator needs the real fields
//   I_b(x) = sum_{m in b} delta(m) exp(+2 pi i m.x / M),  J_b: delta -> 1,
// and, per triangle, sum_x I_b1 I_b2 I_b3 / sum_x J_b1 J_b2 J_b3.  Every mode
// of shells 1..n_bins has |m_a| <= R, so on a grid of M > 3R points per axis
// m1 + m2 + m3 = 0 mod M only when m1 + m2 + m3 = 0: the sums on that grid
// count exactly the closed triplets, as the FFT grid does under the triangle
// limit k < k_f N / 3 of Sec. 4.1.  M is the smallest 2^a 3^b 5^c above 3R
// (800 for 128 shells of 2 k_f), which is never above N.
//
// Design (gfx950).  The n_bins fields of an M^3 grid do not fit in HBM
// (128 x 2 GB at M = 800; the paper notes the N_k x N_G^3 memory of the
// method), so the grid is processed in slabs of S x-planes:
//  1. the modes |m_a| <= R of delta are gathered once into a dense cube
//     (eq. intdelta combination and window deconvolution, as for P(k));
//  2. per slab, a direct DFT along x takes every shell pair q (shells 2q+1 as
//     the real and 2q+2 as the imaginary part of one complex field) from the
//     cube to (x in slab, m_y, m_z): a thread owns one (q, m_y, m_z) and runs
//     over the few m_x of its pair's shells, with exact table twiddles;
//  3. inverse FFTs along z (only the rows |m_y| <= R carry data) and along y
//     give I_2q+1 + i I_2q+2 on the slab's points;
//  4. the triple sums are a dense contraction over points: for a fixed
//     d = b1 - b2, T(b2, b3) = sum_p (I_b1 I_b2)(p) I_b3(p), which MFMA
//     f32 16x16x4 instructions evaluate on tiles of 16 consecutive b2 by 16
//     consecutive b3 ("jobs"; 996 jobs cover the 185,056 closed triangles of
//     128 shells).  A workgroup stages 64-point chunks of every field in LDS
//     and each wave keeps 16 jobs' accumulators in registers: FP32 products
//     and sums over a chunk, FP64 across chunks;
//  5. per-workgroup sums are reduced in a fixed order, slab after slab.
// The J sums depend only on (M, n_dk, n_bins, the jobs) and are cached by the
// caller (api.hip) after the first call.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "modes.hpp"

namespace fsest {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kBsMaxS = 32;          // x planes per slab, at most
constexpr int kBsWaves = 8;          // waves of a triple-sum workgroup
constexpr int kBsJobsPerWave = 16;   // 16x16 tiles whose accumulators a wave holds
constexpr int kBsJobsPerGroup = kBsWaves * kBsJobsPerWave;
constexpr int kBsTargetBlocks = 1024;  // triple-sum workgroups per slab, about
constexpr size_t kBsSlabBudget = (size_t)8 << 30;  // bytes of one slab's fields, at most

// ------------------------------------------------------------------ plan (host)
static bool smooth235_len(int v) {
  if (v < 1) return false;
  for (int p : {2, 3, 5})
    while (v % p == 0) v /= p;
  return v == 1;
}

static size_t bs_align(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t bs_max_jobs(int n_bins) {
  int64_t total = 0;
  for (int d = 0; d < n_bins; ++d) {
    const int bs = d > 0 ? d : 1;
    if (n_bins - d < bs) continue;
    const int64_t r = (n_bins - d - bs) / 16;
    total += (r + 1) * (r + 2) / 2;
  }
  return total;
}

bool bs_plan(int n, int n_dk, int n_bins, int64_t njobs, int64_t n_tri, BsPlan* pl) {
  BsPlan p;
  // |m| < (n_bins + 1/2) n_dk for every mode of shells 1..n_bins
  p.R = ((2 * n_bins + 1) * n_dk - 1) / 2;
  p.M = 3 * p.R + 1;
  while (!smooth235_len(p.M)) ++p.M;
  if (p.M > n || p.M > 1024) return false;
  p.Q = (n_bins + 1) / 2;
  const size_t plane = (size_t)p.Q * p.M * p.M * sizeof(float2);
  p.S = 1;
  for (int s = 1; s <= kBsMaxS && s <= p.M; ++s)
    if (p.M % s == 0 && (size_t)s * plane <= kBsSlabBudget) p.S = s;
  p.nslab = p.M / p.S;
  p.pc = p.Q <= 64 ? 64 : (p.Q <= 128 ? 32 : 16);
  p.npts = (int64_t)p.S * p.M * p.M;
  const int64_t chunks = (p.npts + p.pc - 1) / p.pc;
  p.njobs = njobs;
  p.ngroups = (int)((njobs + kBsJobsPerGroup - 1) / kBsJobsPerGroup);
  int64_t nr = (kBsTargetBlocks + p.ngroups - 1) / (p.ngroups > 0 ? p.ngroups : 1);
  if (nr > chunks) nr = chunks;
  p.nranges = (int)(nr > 0 ? nr : 1);
  // workspace: twiddles, the delta cube, one slab, jobs, triangle map,
  // per-workgroup partial sums (bounded for any job count up to njobs), the
  // two running sums
  const int64_t W = 2 * p.R + 1;
  size_t off = 0;
  p.off_tw = off;   off = bs_align(off + (size_t)p.M * sizeof(float2));
  p.off_band = off; off = bs_align(off + (size_t)W * W * W * sizeof(float2));
  p.off_slab = off; off = bs_align(off + (size_t)p.S * plane);
  p.off_jobs = off; off = bs_align(off + (size_t)njobs * 4 * sizeof(int32_t));
  p.off_tmap = off; off = bs_align(off + (size_t)n_tri * 2 * sizeof(int32_t));
  int64_t part_entries = (int64_t)kBsTargetBlocks * kBsJobsPerGroup + njobs;
  if (part_entries > chunks * njobs) part_entries = chunks * njobs;
  p.off_part = off; off = bs_align(off + (size_t)part_entries * 256 * sizeof(double));
  p.off_run = off;  off = bs_align(off + (size_t)2 * njobs * 256 * sizeof(double));
  p.bytes = off;
  *pl = p;
  return true;
}

void bs_jobs(const int32_t* tri, int64_t n_tri, std::vector<int32_t>& jobs,
             std::vector<int32_t>& tmap) {
  // key (d, r0, c0): rows b2 = bs + 16 r0 + i, columns b3 = bs + 16 c0 + j,
  // bs = max(d, 1); sorted, so consecutive jobs share their row tile
  std::vector<int64_t> keys(n_tri);
  for (int64_t t = 0; t < n_tri; ++t) {
    const int b1 = tri[3 * t], b2 = tri[3 * t + 1], b3 = tri[3 * t + 2];
    const int d = b1 - b2, bs = d > 0 ? d : 1;
    keys[t] = ((int64_t)d * 64 + (b2 - bs) / 16) * 64 + (b3 - bs) / 16;
  }
  std::vector<int64_t> uniq(keys);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  jobs.resize(uniq.size() * 4);
  for (size_t j = 0; j < uniq.size(); ++j) {
    const int64_t k = uniq[j];
    jobs[4 * j + 0] = (int32_t)(k / 4096);
    jobs[4 * j + 1] = (int32_t)((k / 64) % 64);
    jobs[4 * j + 2] = (int32_t)(k % 64);
    jobs[4 * j + 3] = 0;
  }
  tmap.resize(2 * n_tri);
  for (int64_t t = 0; t < n_tri; ++t) {
    const int b1 = tri[3 * t], b2 = tri[3 * t + 1], b3 = tri[3 * t + 2];
    const int d = b1 - b2, bs = d > 0 ? d : 1;
    tmap[2 * t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[t]) - uniq.begin());
    tmap[2 * t + 1] = ((b2 - bs) % 16) * 16 + (b3 - bs) % 16;
  }
}

// ------------------------------------------------------------------ kernels
// exp(-2 pi i n / M), computed in float64
__global__ void k_bs_twiddles(int M, float2* tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double s, c;
  sincospi(-2.0 * i / M, &s, &c);
  tw[i] = make_float2((float)c, (float)s);
}

// delta(m) = C(m) / (N_P W(m)) for |m_a| <= R inside shells 1..n_bins (zero
// elsewhere and at m = 0), cube index ((m_z + R) W + m_y + R) W + m_x + R
__global__ __launch_bounds__(256) void k_bs_band(const float2* __restrict__ data, Geom g, int mock,
                                                 int R, int n_dk, int n_bins,
                                                 const float2* __restrict__ phase,
                                                 const float* __restrict__ win1,
                                                 const double* __restrict__ norm,
                                                 float2* __restrict__ band) {
  const int n = g.n, L = g.nz, W = 2 * R + 1;
  const int64_t total = (int64_t)W * W * W;
  const float inv_np = 1.0f / (float)norm[2 * mock];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mx = (int)(e % W) - R, my = (int)((e / W) % W) - R, mz = (int)(e / ((int64_t)W * W)) - R;
    const int m2 = mx * mx + my * my + mz * mz;
    const int b = m2 ? shell_of(m2, n_dk) : 0;
    float2 d = make_float2(0.f, 0.f);
    if (b >= 1 && b <= n_bins) {
      const int x = fft_index(mx, n), y = fft_index(my, n), z = fft_index(mz, n);
      float2 c;
      if (g.npair > 1) {
        c = multi_mode(data, g, mock, mx, my, mz, phase);
      } else {
        const int xm = neg_mod<false>(x, n), ym = neg_mod<false>(y, n);
        const int zz = ((mz % L) + L) % L, zm = neg_mod<false>(zz, L);
        const float2 za = data[complex_index(g, mock, x, y, zz)];
        const float2 zb = data[complex_index(g, mock, xm, ym, zm)];
        c = g.il ? combined_mode<true, false>(za, zb, mx, my, mz, phase, n)
                 : combined_mode<false, false>(za, zb, mx, my, mz, phase, n);
      }
      const float w = win1[x] * win1[y] * win1[z];
      d = cscale(c, inv_np / w);
    }
    band[e] = d;
  }
}

// floor(sqrt(v)) and ceil(sqrt(v)) of a non-negative int
__device__ __forceinline__ int isqrt_floor(int v) {
  int r = (int)sqrtf((float)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Direct DFT along x of shell pair q for the slab's planes x0 .. x0+S-1:
//   F_q(x, m_y, m_z) = sum_{m_x} (S_b1(m) + i S_b2(m)) d(m) exp(+2 pi i m_x x / M),
// b1 = 2q+1, b2 = 2q+2 (if <= n_bins), d = delta (or 1 for the counts), at
// slab index ((q S + x - x0) M + (m_y mod M)) M + (m_z mod M); zero outside
// |m_y|, |m_z| <= R.  One thread per (q, m_y index, m_z index).
__global__ __launch_bounds__(256) void k_bs_xdft(const float2* __restrict__ band, int R, int M,
                                                 int S, int x0, int Q, int n_dk, int n_bins,
                                                 int counts, const float2* __restrict__ twm,
                                                 float2* __restrict__ slab) {
  __shared__ float2 tw[1024];
  for (int i = threadIdx.x; i < M; i += blockDim.x) tw[i] = twm[i];
  __syncthreads();
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)Q * M * M) return;
  const int bz = (int)(tid % M), ay = (int)((tid / M) % M), q = (int)(tid / ((int64_t)M * M));
  const int my = ay <= M / 2 ? ay : ay - M, mz = bz <= M / 2 ? bz : bz - M;
  float2 acc[kBsMaxS];
#pragma unroll
  for (int xl = 0; xl < kBsMaxS; ++xl) acc[xl] = make_float2(0.f, 0.f);
  if (my >= -R && my <= R && mz >= -R && mz <= R) {
    const int b1 = 2 * q + 1, bhi = (2 * q + 2 <= n_bins) ? 2 * q + 2 : b1;
    const int W = 2 * R + 1;
    const int rho2 = my * my + mz * mz;
    // candidate |m_x|: (2 b1 - 1)^2 n^2 <= 4 m^2 < (2 bhi + 1)^2 n^2, one
    // more on each side, then every candidate is tested with shell_of
    const int lo4 = (2 * b1 - 1) * (2 * b1 - 1) * n_dk * n_dk - 4 * rho2;
    const int hi4 = (2 * bhi + 1) * (2 * bhi + 1) * n_dk * n_dk - 4 * rho2;
    if (hi4 > 0) {
      int umax = isqrt_floor((hi4 - 1) / 4) + 1;
      int umin = lo4 <= 0 ? 0 : isqrt_floor((lo4 + 3) / 4) - 1;
      if (umax > R) umax = R;
      if (umin < 0) umin = 0;
      const float2* row = band + ((int64_t)(mz + R) * W + (my + R)) * W + R;
      for (int u = umin; u <= umax; ++u) {
        const int m2 = u * u + rho2;
        if (m2 == 0) continue;
        const int b = shell_of(m2, n_dk);
        if (b != b1 && b != bhi) continue;
        for (int sg = 0; sg < 2; ++sg) {
          if (u == 0 && sg == 1) continue;
          const int mx = sg ? -u : u;
          float2 d = counts ? make_float2(1.f, 0.f) : row[mx];
          if (b != b1) d = make_float2(-d.y, d.x);  // i d: the imaginary field
          const int step = mx >= 0 ? mx : mx + M;
          int idx = (int)(((int64_t)step * x0) % M);
#pragma unroll
          for (int xl = 0; xl < kBsMaxS; ++xl) {
            if (xl < S) {
              const float2 w = tw[idx];  // exp(-2 pi i idx / M); conjugated below
              acc[xl].x += d.x * w.x + d.y * w.y;
              acc[xl].y += d.y * w.x - d.x * w.y;
              idx += step;
              if (idx >= M) idx -= M;
            }
          }
        }
      }
    }
  }
  float2* out = slab + ((int64_t)q * S * M + ay) * M + bz;
#pragma unroll
  for (int xl = 0; xl < kBsMaxS; ++xl)
    if (xl < S) out[(int64_t)xl * M * M] = acc[xl];
}

// Triple sums of one slab.  Fields: pair q at slab + q npts, point p, real
// part field 2q (shell 2q+1), imaginary part field 2q+1 (shell 2q+2).  A job
// (d, r0, c0) is the 16x16 tile T(i, j) = sum_p I_b1 I_b2 I_b3 with
// b2 = bs + 16 r0 + i, b1 = b2 + d, b3 = bs + 16 c0 + j, bs = max(d, 1)
// (shells above n_bins read a zero row).  Workgroup = (point range, job
// group); wave w of the group owns jobs g 128 + 16 w .. + 15.  MFMA
// v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16] in register r; lane
// l's four K-slots of the PC/4 steps are the points (l / 16) PC/4 + s.
template <int PC>
__global__ __launch_bounds__(kBsWaves * 64) void k_bs_triple(
    const float2* __restrict__ slab, int64_t npts, int Q, int n_bins,
    const int32_t* __restrict__ jobs, int njobs, int ngroups, int nranges,
    double* __restrict__ partial) {
  constexpr int KS = PC / 4;       // MFMA steps per chunk = points per lane
  constexpr int STRIDE = PC + 4;   // floats per field row in LDS
  constexpr int NT = kBsWaves * 64;
  extern __shared__ __align__(16) float fld[];
  const int grp = blockIdx.x % ngroups, rng = blockIdx.x / ngroups;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, i16 = lane & 15, k4 = lane >> 4;
  const int j0 = grp * kBsJobsPerGroup + wave * kBsJobsPerWave;
  const int nj = njobs - j0 < 0 ? 0 : (njobs - j0 > kBsJobsPerWave ? kBsJobsPerWave : njobs - j0);
  double acc[kBsJobsPerWave][4];
#pragma unroll
  for (int jj = 0; jj < kBsJobsPerWave; ++jj)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[jj][r] = 0.0;

  const int64_t nch = (npts + PC - 1) / PC;
  const int64_t cbeg = nch * rng / nranges, cend = nch * (rng + 1) / nranges;
  // the zero row (shells above n_bins)
  for (int t = threadIdx.x; t < STRIDE; t += NT) fld[n_bins * STRIDE + t] = 0.0f;
  // this thread's share of a chunk: elements e = threadIdx.x + NT u of Q x PC
  constexpr int UMAX = (128 * 32 + NT - 1) / NT;  // Q PC <= 4096 by the choice of PC
  const int nel = Q * PC;
  float2 pre[UMAX];
  auto fetch = [&](int64_t c) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int e = threadIdx.x + NT * u;
      pre[u] = make_float2(0.f, 0.f);
      if (e < nel) {
        const int q = e / PC;
        const int64_t p = c * PC + (e % PC);
        if (p < npts) pre[u] = slab[(int64_t)q * npts + p];
      }
    }
  };
  if (cbeg < cend) fetch(cbeg);
  for (int64_t c = cbeg; c < cend; ++c) {
    __syncthreads();  // the previous chunk is consumed
#pragma unroll
    for (int u = 0; u < UMAX; ++u) {
      const int e = threadIdx.x + NT * u;
      if (e < nel) {
        const int q = e / PC, pt = e % PC;
        fld[(2 * q) * STRIDE + pt] = pre[u].x;
        if (2 * q + 1 < n_bins) fld[(2 * q + 1) * STRIDE + pt] = pre[u].y;
      }
    }
    __syncthreads();
    if (c + 1 < cend) fetch(c + 1);
    float a[KS], bv[KS];
    int prev_d = -1, prev_r0 = -1;
#pragma unroll
    for (int jj = 0; jj < kBsJobsPerWave; ++jj) {
      if (jj < nj) {
        // job descriptor (wave-uniform: scalar loads); LDS rows of the A
        // factors (b1, b2) and the B factor (b3) of this lane's row / column,
        // the zero row for shells above n_bins
        const int32_t* jd = jobs + 4 * (j0 + jj);
        const int d = jd[0], r0 = jd[1], c0 = jd[2];
        const int bs = d > 0 ? d : 1;
        if (d != prev_d || r0 != prev_r0) {
          const int b2 = bs + 16 * r0 + i16, b1 = b2 + d;
          const int fa1 = b1 <= n_bins ? b1 - 1 : n_bins, fa2 = b1 <= n_bins ? b2 - 1 : n_bins;
          const float4* r1 = reinterpret_cast<const float4*>(fld + fa1 * STRIDE + k4 * KS);
          const float4* r2 = reinterpret_cast<const float4*>(fld + fa2 * STRIDE + k4 * KS);
#pragma unroll
          for (int v = 0; v < KS / 4; ++v) {
            const float4 x1 = r1[v], x2 = r2[v];
            a[4 * v + 0] = x1.x * x2.x;
            a[4 * v + 1] = x1.y * x2.y;
            a[4 * v + 2] = x1.z * x2.z;
            a[4 * v + 3] = x1.w * x2.w;
          }
          prev_d = d;
          prev_r0 = r0;
        }
        const int b3 = bs + 16 * c0 + i16;
        const int fb = b3 <= n_bins ? b3 - 1 : n_bins;
        const float4* r3 = reinterpret_cast<const float4*>(fld + fb * STRIDE + k4 * KS);
#pragma unroll
        for (int v = 0; v < KS / 4; ++v) {
          const float4 x3 = r3[v];
          bv[4 * v + 0] = x3.x;
          bv[4 * v + 1] = x3.y;
          bv[4 * v + 2] = x3.z;
          bv[4 * v + 3] = x3.w;
        }
        v4f cacc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s) cacc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv[s], cacc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[jj][r] += (double)cacc[r];
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < kBsJobsPerWave; ++jj) {
    if (jj < nj) {
      double* dst = partial + ((int64_t)rng * njobs + j0 + jj) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[(4 * k4 + r) * 16 + i16] = acc[jj][r];
    }
  }
}

// run[j] += sum over point ranges of partial[range][j], ranges in order
__global__ void k_bs_reduce(const double* __restrict__ partial, int64_t entries, int nranges,
                            double* __restrict__ run) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= entries) return;
  double s = 0.0;
  for (int r = 0; r < nranges; ++r) s += partial[(int64_t)r * entries + e];
  run[e] += s;
}

// B = V^2 sum III / sum JJJ (NaN without closed triplets), N_tri = sum JJJ / M^3
__global__ void k_bs_finalize(const int32_t* __restrict__ tmap, int64_t n_tri,
                              const double* __restrict__ run_i, const double* __restrict__ run_j,
                              double vol, double m3, double* __restrict__ bk, double* __restrict__ ntri) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tri) return;
  const int64_t e = (int64_t)tmap[2 * t] * 256 + tmap[2 * t + 1];
  const double si = run_i[e], sj = run_j[e];
  bk[t] = (sj > 0.5) ? vol * vol * si / sj : __builtin_nan("");
  ntri[t] = sj / m3;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_bs_setup(const Geom& g, const Buffers& b, int mock, int n_dk, int n_bins,
                           const BsPlan& pl, char* bws, hipStream_t s) {
  float2* tw = (float2*)(bws + pl.off_tw);
  float2* band = (float2*)(bws + pl.off_band);
  hipLaunchKernelGGL(k_bs_twiddles, dim3((pl.M + 255) / 256), dim3(256), 0, s, pl.M, tw);
  const int64_t W = 2 * pl.R + 1;
  const int64_t total = W * W * W;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_bs_band, dim3(blocks), dim3(256), 0, s, (const float2*)b.grid, g, mock, pl.R,
                     n_dk, n_bins, b.phase, b.win1, b.norm, band);
  return hipGetLastError();
}

template <int PC>
static hipError_t triple_t(const BsPlan& pl, const float2* slab, int n_bins, const int32_t* jobs,
                           double* part, hipStream_t s) {
  const size_t lds = sizeof(float) * (size_t)(n_bins + 1) * (PC + 4);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_bs_triple<PC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_bs_triple<PC>), dim3((unsigned)(pl.ngroups * pl.nranges)),
                     dim3(kBsWaves * 64), lds, s, slab, pl.npts, pl.Q, n_bins, jobs, (int)pl.njobs,
                     pl.ngroups, pl.nranges, part);
  return hipGetLastError();
}

hipError_t launch_bs_fields(int n_dk, int n_bins, const BsPlan& pl, char* bws, bool counts, int slab_index,
                            hipStream_t s) {
  const float2* tw = (const float2*)(bws + pl.off_tw);
  const float2* band = (const float2*)(bws + pl.off_band);
  float2* slab = (float2*)(bws + pl.off_slab);
  const int M = pl.M, R = pl.R;
  const int64_t plane = (int64_t)M * M;
  const int64_t xthreads = (int64_t)pl.Q * plane;
  hipLaunchKernelGGL(k_bs_xdft, dim3((unsigned)((xthreads + 255) / 256)), dim3(256), 0, s, band, R, M,
                     pl.S, slab_index * pl.S, pl.Q, n_dk, n_bins, counts ? 1 : 0, tw, slab);
  // inverse z transforms of the rows that carry data (|m_y| <= R), then y
  const int64_t planes = (int64_t)pl.Q * pl.S;
  hipError_t e = launch_fft_rows_len(M, slab, planes * (R + 1), R + 1, plane, +1, tw, s);
  if (e != hipSuccess) return e;
  if (R > 0 &&
      (e = launch_fft_rows_len(M, slab + (int64_t)(M - R) * M, planes * R, R, plane, +1, tw, s)) !=
          hipSuccess)
    return e;
  return launch_fft_cols_len(M, slab, M, M, planes, plane, +1, 16, tw, s);
}

hipError_t launch_bs_triple(int n_bins, const BsPlan& pl, char* bws, bool first_slab, double* run,
                            hipStream_t s) {
  const float2* slab = (const float2*)(bws + pl.off_slab);
  const int32_t* jobs = (const int32_t*)(bws + pl.off_jobs);
  double* part = (double*)(bws + pl.off_part);
  const int64_t entries = pl.njobs * 256;
  hipError_t e = hipSuccess;
  if (first_slab && (e = launch_fill_u32((uint32_t*)run, (size_t)entries * 2, 0u, s)) != hipSuccess)
    return e;
  if (pl.pc == 64) e = triple_t<64>(pl, slab, n_bins, jobs, part, s);
  else if (pl.pc == 32) e = triple_t<32>(pl, slab, n_bins, jobs, part, s);
  else e = triple_t<16>(pl, slab, n_bins, jobs, part, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bs_reduce, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s, part,
                     entries, pl.nranges, run);
  return hipGetLastError();
}

hipError_t launch_bs_finalize(const BsPlan& pl, char* bws, int64_t n_tri, double vol, double* bk,
                              double* ntri, hipStream_t s) {
  const int32_t* tmap = (const int32_t*)(bws + pl.off_tmap);
  const double* run = (const double*)(bws + pl.off_run);
  const double m3 = (double)pl.M * pl.M * pl.M;
  hipLaunchKernelGGL(k_bs_finalize, dim3((unsigned)((n_tri + 255) / 256)), dim3(256), 0, s, tmap,
                     n_tri, run, run + pl.njobs * 256, vol, m3, bk, ntri);
  return hipGetLastError();
}

}  // namespace fsest
