// Mass assignment (Sec. 2.3, eq. delgrid) onto the primary grid and the grid
// shifted by H/2 on every axis (Sec. 3.1), and its adjoint gather.
//
// Design (gfx950): particles are counting-sorted by bucket (kBucket^3 cells)
// so that every deposit workgroup owns one output tile of T^3 cells outright:
// it reads the particles of the buckets that can reach the tile, adds the
// clipped footprints of both grids with LDS float atomics, and writes the
// finished tile once with coalesced stores.  No global atomics touch the grid
// and the grid needs no clearing.  A particle whose base cell is c reaches
// cells c-1 .. c+3 of either grid for every p <= 4, so the buckets holding
// cells t0-3 .. t0+T are enough.
#include <type_traits>

#include "fsest_internal.hpp"

namespace fsest {

// ------------------------------------------------------------------ utils
__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_set_counts(const int64_t* offsets, int64_t n_total, int batch, int64_t* np) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  np[i] = offsets ? (offsets[i + 1] - offsets[i]) : n_total;
}

hipError_t launch_set_counts(const int64_t* offsets, int64_t n_total, int batch, int64_t* np,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_set_counts, dim3((batch + 63) / 64), dim3(64), 0, s, offsets, n_total,
                     batch, np);
  return hipGetLastError();
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

__device__ __forceinline__ int base_cell(double u, int n) {
  return ((int)floor(u)) & (n - 1);
}

// ------------------------------------------------------------------ sort
template <typename TP>
__global__ __launch_bounds__(256) void k_bucket_count(const TP* __restrict__ pos, int64_t n_total,
                                                      const int64_t* __restrict__ offsets, Geom g,
                                                      uint32_t* __restrict__ counts,
                                                      uint32_t* __restrict__ rank) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  double x, y, z;
  load_pos(pos, j, x, y, z);
  const int mock = mock_of(offsets, g.batch, j);
  const int bx = base_cell(grid_coord(x, g.box, g.inv), g.n) / kBucket;
  const int by = base_cell(grid_coord(y, g.box, g.inv), g.n) / kBucket;
  const int bz = base_cell(grid_coord(z, g.box, g.inv), g.n) / kBucket;
  const uint32_t key = (uint32_t)(((int64_t)mock * g.nb + bx) * g.nb + by) * g.nb + bz;
  rank[j] = atomicAdd(&counts[key], 1u);
}

template <typename TP>
__global__ __launch_bounds__(256) void k_bucket_scatter(const TP* __restrict__ pos, int64_t n_total,
                                                        const int64_t* __restrict__ offsets, Geom g,
                                                        const uint32_t* __restrict__ boff,
                                                        const uint32_t* __restrict__ rank,
                                                        TP* __restrict__ sorted) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  TP px = pos[3 * j + 0], py = pos[3 * j + 1], pz = pos[3 * j + 2];
  const int mock = mock_of(offsets, g.batch, j);
  const int bx = base_cell(grid_coord((double)px, g.box, g.inv), g.n) / kBucket;
  const int by = base_cell(grid_coord((double)py, g.box, g.inv), g.n) / kBucket;
  const int bz = base_cell(grid_coord((double)pz, g.box, g.inv), g.n) / kBucket;
  const uint32_t key = (uint32_t)(((int64_t)mock * g.nb + bx) * g.nb + by) * g.nb + bz;
  const int64_t dst = (int64_t)boff[key] + rank[j];
  sorted[3 * dst + 0] = px;
  sorted[3 * dst + 1] = py;
  sorted[3 * dst + 2] = pz;
}

// exclusive scan of n items in place, 2048 items per block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  // Hillis-Steele over the block in LDS (256 entries)
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    uint32_t a = (t >= off) ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(uint32_t* data, size_t n, uint32_t* sums,
                                                           uint32_t* maxcount) {
  __shared__ uint32_t sh[kScanThreads];
  const size_t base = (size_t)blockIdx.x * kScanBlock + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t run = 0, mx = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? data[base + i] : 0u;
    uint32_t c = v[i];
    mx = max(mx, c);
    v[i] = run;
    run += c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_down((int)mx, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(maxcount, mx);
  uint32_t total;
  uint32_t pre = block_exclusive_scan(run, sh, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) data[base + i] = v[i] + pre;
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t* sums, int nblk) {
  __shared__ uint32_t sh[kScanThreads];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nblk; c0 += kScanThreads) {
    int i = c0 + threadIdx.x;
    uint32_t v = (i < nblk) ? sums[i] : 0u;
    uint32_t total;
    uint32_t pre = block_exclusive_scan(v, sh, total);
    if (i < nblk) sums[i] = pre + carry;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t* data, size_t n, const uint32_t* sums) {
  const uint32_t add = sums[blockIdx.x];
  const size_t base = (size_t)blockIdx.x * kScanBlock;
  for (int i = threadIdx.x; i < kScanBlock; i += kScanThreads)
    if (base + i < n) data[base + i] += add;
}

hipError_t launch_sort(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                       int64_t n_total, const Buffers& b, hipStream_t s) {
  const size_t nkeys = (size_t)g.batch * g.nb * g.nb * g.nb;
  hipError_t e = launch_fill_u32(b.boff, nkeys + 1, 0u, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(b.stats, 1, 0u, s)) != hipSuccess) return e;
  const unsigned pblocks = (unsigned)((n_total + 255) / 256);
  if (dt == EST_F32)
    hipLaunchKernelGGL(k_bucket_count<float>, dim3(pblocks), dim3(256), 0, s, (const float*)pos,
                       n_total, offsets, g, b.boff, b.rank);
  else
    hipLaunchKernelGGL(k_bucket_count<double>, dim3(pblocks), dim3(256), 0, s, (const double*)pos,
                       n_total, offsets, g, b.boff, b.rank);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t n = nkeys + 1;
  const int nblk = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nblk), dim3(kScanThreads), 0, s, b.boff, n, b.scan_tmp,
                     b.stats);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, b.scan_tmp, nblk);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk), dim3(kScanThreads), 0, s, b.boff, n, b.scan_tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (dt == EST_F32)
    hipLaunchKernelGGL(k_bucket_scatter<float>, dim3(pblocks), dim3(256), 0, s, (const float*)pos,
                       n_total, offsets, g, b.boff, b.rank, (float*)b.sorted);
  else
    hipLaunchKernelGGL(k_bucket_scatter<double>, dim3(pblocks), dim3(256), 0, s,
                       (const double*)pos, n_total, offsets, g, b.boff, b.rank,
                       (double*)b.sorted);
  return hipGetLastError();
}

// ------------------------------------------------------------------ stencils
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
  } else {
    const float t = 1.0f - f;
    const float f2 = f * f, t2 = t * t;
    w[0] = t2 * t * (1.0f / 6.0f);
    w[1] = (4.0f - 6.0f * f2 + 3.0f * f2 * f) * (1.0f / 6.0f);
    w[2] = (4.0f - 6.0f * t2 + 3.0f * t2 * t) * (1.0f / 6.0f);
    w[3] = f2 * f * (1.0f / 6.0f);
  }
#pragma unroll
  for (int i = 0; i < P; ++i) cell[i] = (first + i) & (n - 1);
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

// ------------------------------------------------------------------ deposit
// Fixed-point accumulation.  LDS float atomics are ~20x slower than integer
// ones on gfx950, so a workgroup sums its tile in unsigned integers: a weight
// product w in [0, 1] adds round(w * S).  Two formats:
//  * wide (64-bit): S = 2^32 - 2^8; a grid sums to N_P < 2^31 units, so no
//    cell can overflow;
//  * narrow (32-bit): S = 2^F with F chosen on the device from the largest
//    bucket count M of this deposit.  A cell only receives particles whose
//    base cell lies in a 5^3 block, which meets at most 8 buckets, so its sum
//    is at most B = 8 M units plus half a unit per contribution; F is the
//    largest value with B (2^F + 1) < 2^32.  When F < 24 (coarser than the
//    float32 resolution of a unit weight) the wide kernel runs
//    instead (both are launched; the one not selected returns at once).
// Integer sums are exact, so deposits are bitwise reproducible.
constexpr float kFixWide = 4294967040.0f;  // 2^32 - 2^8
constexpr int kNarrowMinBits = 24;
constexpr int kListCap = 2048;  // LDS list of particles that reach the tile

__device__ __forceinline__ int narrow_bits(uint32_t maxcount) {
  const double bound = 8.0 * (double)(maxcount > 0 ? maxcount : 1);
  int f = 0;
  while (f < 31 && bound * (ldexp(1.0, f + 1) + 1.0) < 4294967295.0) ++f;
  return f;
}

struct DepRanges {
  uint32_t start[72];
  uint32_t pref[73];
  int count;
};

// does the reach c-1 .. c+3 (both grids, every p <= 4) of base cell c touch
// [t0, t0 + T) on a periodic axis of length n?
__device__ __forceinline__ bool axis_reaches(int c, int t0, int T, int n) {
  const int lo = (c - 1 - t0) & (n - 1);
  return lo < T || lo > n - 5;
}

// ... and does it lie inside [t0, t0 + T)?
__device__ __forceinline__ bool axis_inside(int c, int t0, int T, int n) {
  const int lo = (c - 1 - t0) & (n - 1);
  return T == n || lo <= T - 5;
}

// Adds one particle's footprint (both grids) to the tile.  INTERIOR: the
// footprint is known to lie inside the tile (no masks).  Otherwise cells
// outside the tile are skipped, either by branches or (BRANCHFREE) by adding
// 0 to this lane's own dummy slot acc[dummy].
template <int P, bool IL, typename TP, typename AT, bool INTERIOR, bool BRANCHFREE>
__device__ __forceinline__ void deposit_particle(const TP* __restrict__ sorted, uint32_t j, const Geom& g,
                                                 int t0x, int t0y, int t0z, int T, AT* acc,
                                                 int dummy, float scale) {
  constexpr int NG = IL ? 2 : 1;
  const int n = g.n;
  const int T3 = T * T * T;
  double x, y, z;
  load_pos(sorted, (int64_t)j, x, y, z);
  const double ux = grid_coord(x, g.box, g.inv);
  const double uy = grid_coord(y, g.box, g.inv);
  const double uz = grid_coord(z, g.box, g.inv);
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    const double sh = gi ? 0.5 : 0.0;
    int cx[P], cy[P], cz[P];
    float wx[P], wy[P], wz[P];
    stencil_1d<P>(ux + sh, n, cx, wx);
    stencil_1d<P>(uy + sh, n, cy, wy);
    stencil_1d<P>(uz + sh, n, cz, wz);
    int lx[P], ly[P], lz[P];
    bool ix[P], iy[P], iz[P];
    unsigned mx = 0, my = 0, mz = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      lx[i] = (cx[i] - t0x) & (n - 1);
      ly[i] = (cy[i] - t0y) & (n - 1);
      lz[i] = (cz[i] - t0z) & (n - 1);
      ix[i] = lx[i] < T;
      iy[i] = ly[i] < T;
      iz[i] = lz[i] < T;
      mx |= ix[i] ? (1u << i) : 0u;
      my |= iy[i] ? (1u << i) : 0u;
      mz |= iz[i] ? (1u << i) : 0u;
    }
    if constexpr (!INTERIOR && !BRANCHFREE)
      if (!mx || !my || !mz) continue;
    const int base = gi * T3;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      if constexpr (!INTERIOR && !BRANCHFREE)
        if (!(mx & (1u << i))) continue;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if constexpr (!INTERIOR && !BRANCHFREE)
          if (!(my & (1u << k))) continue;
        const float wxy = wx[i] * wy[k] * scale;
        const int rowi = base + (lx[i] * T + ly[k]) * T;
#pragma unroll
        for (int l = 0; l < P; ++l) {
          if constexpr (INTERIOR) {
            atomicAdd(&acc[rowi + lz[l]], (AT)__float2uint_rn(wxy * wz[l]));
          } else if constexpr (BRANCHFREE) {
            const bool in = ix[i] && iy[k] && iz[l];
            const unsigned q = in ? __float2uint_rn(wxy * wz[l]) : 0u;
            atomicAdd(&acc[in ? rowi + lz[l] : dummy], (AT)q);
          } else {
            if (!(mz & (1u << l))) continue;
            atomicAdd(&acc[rowi + lz[l]], (AT)__float2uint_rn(wxy * wz[l]));
          }
        }
      }
    }
  }
}

template <int P, bool IL, typename TP, bool WIDE, bool BRANCHFREE>
__global__ __launch_bounds__(1024) void k_deposit(const TP* __restrict__ sorted,
                                                  const uint32_t* __restrict__ boff, float* grid,
                                                  Geom g, const uint32_t* __restrict__ stats,
                                                  int exclusive) {
  using AT = typename std::conditional<WIDE, unsigned long long, unsigned>::type;
  constexpr int TM = kTileMax;
  constexpr int NG = IL ? 2 : 1;
  constexpr int MAXW = 16;  // waves per workgroup (1024 threads)
  __shared__ AT acc[NG * TM * TM * TM + 64];  // + one dummy slot per lane
  __shared__ DepRanges rg;
  __shared__ uint32_t list[kListCap];
  __shared__ int wave_cnt[2 * MAXW];
  __shared__ int fill_in, fill_edge;

  // fixed-point format for this deposit (uniform over the grid)
  const int nbits = narrow_bits(stats[0]);
  if (!WIDE && nbits < kNarrowMinBits) return;          // the wide kernel does it
  if (WIDE && !exclusive && nbits >= kNarrowMinBits) return;  // the narrow one does it
  const float scale = WIDE ? kFixWide : ldexpf(1.0f, nbits);
  const double inv_scale = 1.0 / (double)scale;

  const int n = g.n, T = g.tile, nb = g.nb;
  const int tpa = n / T;  // tiles per axis
  const int64_t tid_all = blockIdx.x;
  const int mock = (int)(tid_all / ((int64_t)tpa * tpa * tpa));
  const int trem = (int)(tid_all % ((int64_t)tpa * tpa * tpa));
  const int tx = trem / (tpa * tpa), ty = (trem / tpa) % tpa, tz = trem % tpa;
  const int t0x = tx * T, t0y = ty * T, t0z = tz * T;
  const int T3 = T * T * T;
  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (nthreads + 63) >> 6;

  for (int i = threadIdx.x; i < NG * T3 + 64; i += nthreads) acc[i] = 0;
  if (threadIdx.x == 0) {
    fill_in = 0;
    fill_edge = 0;
  }

  // bucket neighbourhood: buckets of cells t0-3 .. t0+T, or every bucket
  int cnt = T / kBucket + 2;
  if (cnt > nb) cnt = nb;
  const int b0x = (cnt == nb) ? 0 : (t0x / kBucket - 1 + nb) % nb;
  const int b0y = (cnt == nb) ? 0 : (t0y / kBucket - 1 + nb) % nb;
  const int b0z = (cnt == nb) ? 0 : (t0z / kBucket - 1 + nb) % nb;
  const int ncomb = cnt * cnt;  // <= 36
  const int64_t mbase = (int64_t)mock * nb * nb * nb;
  if (wave == 0) {
    uint32_t s0 = 0, e0 = 0, s1 = 0, e1 = 0;
    if (lane < ncomb) {
      const int ix = lane / cnt, iy = lane % cnt;
      const int bx = (b0x + ix) % nb, by = (b0y + iy) % nb;
      const int64_t row = mbase + ((int64_t)bx * nb + by) * nb;
      const int z1 = b0z + cnt;  // exclusive end, may exceed nb (wrap)
      if (z1 <= nb) {
        s0 = boff[row + b0z];
        e0 = boff[row + z1];
      } else {
        s0 = boff[row + b0z];
        e0 = boff[row + nb];
        s1 = boff[row];
        e1 = boff[row + (z1 - nb)];
      }
    }
    // exclusive prefix of the per-lane lengths across the wave
    const uint32_t la = e0 - s0, lb = e1 - s1;
    uint32_t incl = la + lb;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)incl, off, 64);
      if (lane >= off) incl += o;
    }
    const uint32_t excl = incl - la - lb;
    if (lane < ncomb) {
      rg.start[2 * lane] = s0;
      rg.start[2 * lane + 1] = s1;
      rg.pref[2 * lane + 1] = excl + la;
      rg.pref[2 * lane + 2] = excl + la + lb;
    }
    if (lane == 0) {
      rg.pref[0] = 0;
      rg.count = 2 * ncomb;
    }
  }
  __syncthreads();
  const uint32_t total = rg.pref[rg.count];
  const int nr = rg.count;

  // rounds of nthreads items: particles that reach the tile go to an LDS
  // list (fully inside ones from the front, the others from the back); the
  // list is deposited whenever another round might not fit
  for (uint32_t r0 = 0; r0 < total; r0 += nthreads) {
    const uint32_t item = r0 + threadIdx.x;
    bool useful = false, inside = false;
    uint32_t j = 0;
    if (item < total) {
      int lo = 0, hi = nr;  // pref[lo] <= item < pref[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rg.pref[mid] <= item) lo = mid; else hi = mid;
      }
      j = rg.start[lo] + (item - rg.pref[lo]);
      double x, y, z;
      load_pos(sorted, (int64_t)j, x, y, z);
      const int cx = base_cell(grid_coord(x, g.box, g.inv), n);
      const int cy = base_cell(grid_coord(y, g.box, g.inv), n);
      const int cz = base_cell(grid_coord(z, g.box, g.inv), n);
      useful = axis_reaches(cx, t0x, T, n) && axis_reaches(cy, t0y, T, n) &&
               axis_reaches(cz, t0z, T, n);
      inside = useful && axis_inside(cx, t0x, T, n) && axis_inside(cy, t0y, T, n) &&
               axis_inside(cz, t0z, T, n);
    }
    const bool edge = useful && !inside;
    const unsigned long long bal_in = __ballot(inside);
    const unsigned long long bal_ed = __ballot(edge);
    if (lane == 0) {
      wave_cnt[wave] = __popcll(bal_in);
      wave_cnt[MAXW + wave] = __popcll(bal_ed);
    }
    __syncthreads();
    int before_in = 0, before_ed = 0, tot_in = 0, tot_ed = 0;
    for (int w = 0; w < nwaves; ++w) {
      const int ci = wave_cnt[w], ce = wave_cnt[MAXW + w];
      before_in += (w < wave) ? ci : 0;
      before_ed += (w < wave) ? ce : 0;
      tot_in += ci;
      tot_ed += ce;
    }
    const int fi0 = fill_in, fe0 = fill_edge;
    const unsigned long long below = (1ull << lane) - 1ull;
    if (inside) list[fi0 + before_in + __popcll(bal_in & below)] = j;
    if (edge) list[kListCap - 1 - (fe0 + before_ed + __popcll(bal_ed & below))] = j;
    __syncthreads();
    const int fi = fi0 + tot_in, fe = fe0 + tot_ed;
    const bool last = r0 + nthreads >= total;
    if (fi + fe > kListCap - nthreads || last) {
      for (int e = threadIdx.x; e < fi; e += nthreads)
        deposit_particle<P, IL, TP, AT, true, false>(sorted, list[e], g, t0x, t0y, t0z, T, acc,
                                                     NG * T3 + lane, scale);
      for (int e = threadIdx.x; e < fe; e += nthreads)
        deposit_particle<P, IL, TP, AT, false, BRANCHFREE>(sorted, list[kListCap - 1 - e], g, t0x,
                                                           t0y, t0z, T, acc, NG * T3 + lane, scale);
      __syncthreads();
      if (threadIdx.x == 0) {
        fill_in = 0;
        fill_edge = 0;
      }
    } else if (threadIdx.x == 0) {
      fill_in = fi;
      fill_edge = fe;
    }
    __syncthreads();
  }

  for (int i = threadIdx.x; i < T3; i += nthreads) {
    const int lx = i / (T * T), ly = (i / T) % T, lz = i % T;
    const float v1 = (float)((double)acc[i] * inv_scale);
    if constexpr (IL) {
      const float v2 = (float)((double)acc[T3 + i] * inv_scale);
      reinterpret_cast<float2*>(grid)[complex_index(g, mock, t0x + lx, t0y + ly, t0z + lz)] =
          make_float2(v1, v2);
    } else {
      grid[real_cell_index(g, mock, t0x + lx, t0y + ly, t0z + lz)] = v1;
    }
  }
}

template <int P, bool IL, typename TP, bool BF>
static void deposit_launch(const Geom& g, const Buffers& b, int threads, bool narrow, hipStream_t s) {
  const int tpa = g.n / g.tile;
  const unsigned blocks = (unsigned)((int64_t)g.batch * tpa * tpa * tpa);
  if (narrow)
    hipLaunchKernelGGL((k_deposit<P, IL, TP, false, BF>), dim3(blocks), dim3(threads), 0, s,
                       (const TP*)b.sorted, b.boff, (float*)b.grid, g, b.stats, 0);
  hipLaunchKernelGGL((k_deposit<P, IL, TP, true, BF>), dim3(blocks), dim3(threads), 0, s,
                     (const TP*)b.sorted, b.boff, (float*)b.grid, g, b.stats, narrow ? 0 : 1);
}

template <int P, bool IL>
static void dispatch_deposit_t(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                               int threads, hipStream_t s) {
  const bool narrow = tu.dep_narrow != 0;
  if (dt == EST_F32) {
    if (tu.dep_branchfree) deposit_launch<P, IL, float, true>(g, b, threads, narrow, s);
    else deposit_launch<P, IL, float, false>(g, b, threads, narrow, s);
  } else {
    if (tu.dep_branchfree) deposit_launch<P, IL, double, true>(g, b, threads, narrow, s);
    else deposit_launch<P, IL, double, false>(g, b, threads, narrow, s);
  }
}

template <int P>
static void dispatch_deposit_p(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                               int threads, hipStream_t s) {
  if (g.il) dispatch_deposit_t<P, true>(g, dt, b, tu, threads, s);
  else dispatch_deposit_t<P, false>(g, dt, b, tu, threads, s);
}

hipError_t launch_deposit(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                          hipStream_t s) {
  int threads = tu.dep_threads;
  if (threads != 256 && threads != 512 && threads != 1024) threads = 1024;
  switch (g.order) {
    case 1: dispatch_deposit_p<1>(g, dt, b, tu, threads, s); break;
    case 2: dispatch_deposit_p<2>(g, dt, b, tu, threads, s); break;
    case 3: dispatch_deposit_p<3>(g, dt, b, tu, threads, s); break;
    default: dispatch_deposit_p<4>(g, dt, b, tu, threads, s); break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ test hook
__global__ void k_copy_grid(const float* grid, Geom g, int which, int mock, float* dst) {
  const int n = g.n;
  const int64_t n3 = (int64_t)n * n * n;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n3; i += stride) {
    const int x = (int)(i / ((int64_t)n * n)), y = (int)((i / n) % n), z = (int)(i % n);
    if (g.il)
      dst[i] = grid[2 * complex_index(g, mock, x, y, z) + (which - 1)];
    else
      dst[i] = grid[real_cell_index(g, mock, x, y, z)];
  }
}

hipError_t launch_copy_grid(const Geom& g, const Buffers& b, int which, int mock, float* dst,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_copy_grid, dim3(4096), dim3(256), 0, s, (const float*)b.grid, g, which,
                     mock, dst);
  return hipGetLastError();
}

// ------------------------------------------------------------------ adjoint gather
// dL/dx_{j,alpha} = -(N/L) sum_a sum_{g in stencil_a} G_a(g) W'(s_alpha) prod_{beta != alpha} W(s_beta)
// where G_a = dL/drho_a sits in the grid buffer with the deposit's layout.
template <int P, bool IL, typename TP>
__global__ __launch_bounds__(256) void k_gather_grad(const TP* __restrict__ pos, int64_t n_total,
                                                     const int64_t* __restrict__ offsets,
                                                     const float* __restrict__ grid, Geom g,
                                                     TP* __restrict__ grad) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  double x, y, z;
  load_pos(pos, j, x, y, z);
  const int mock = mock_of(offsets, g.batch, j);
  const int n = g.n;
  const double u[3] = {grid_coord(x, g.box, g.inv), grid_coord(y, g.box, g.inv),
                       grid_coord(z, g.box, g.inv)};
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  constexpr int NG = IL ? 2 : 1;
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    const double sh = gi ? 0.5 : 0.0;
    int c[3][P];
    float w[3][P], d[3][P];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      stencil_1d<P>(u[ax] + sh, n, c[ax], w[ax]);
      stencil_1d_deriv<P>(u[ax] + sh, d[ax]);
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
      for (int bq = 0; bq < P; ++bq) {
#pragma unroll
        for (int cq = 0; cq < P; ++cq) {
          const float gv = IL ? grid[2 * complex_index(g, mock, c[0][a], c[1][bq], c[2][cq]) + gi]
                              : grid[real_cell_index(g, mock, c[0][a], c[1][bq], c[2][cq])];
          gx += gv * d[0][a] * w[1][bq] * w[2][cq];
          gy += gv * w[0][a] * d[1][bq] * w[2][cq];
          gz += gv * w[0][a] * w[1][bq] * d[2][cq];
        }
      }
    }
  }
  const double sc = -(double)n / g.box;
  grad[3 * j + 0] = (TP)(sc * gx);
  grad[3 * j + 1] = (TP)(sc * gy);
  grad[3 * j + 2] = (TP)(sc * gz);
}

template <int P>
static void dispatch_gather(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                            int64_t n_total, const Buffers& b, void* grad, hipStream_t s) {
  const unsigned blocks = (unsigned)((n_total + 255) / 256);
  if (dt == EST_F32) {
    if (g.il)
      hipLaunchKernelGGL((k_gather_grad<P, true, float>), dim3(blocks), dim3(256), 0, s,
                         (const float*)pos, n_total, offsets, (const float*)b.grid, g, (float*)grad);
    else
      hipLaunchKernelGGL((k_gather_grad<P, false, float>), dim3(blocks), dim3(256), 0, s,
                         (const float*)pos, n_total, offsets, (const float*)b.grid, g, (float*)grad);
  } else {
    if (g.il)
      hipLaunchKernelGGL((k_gather_grad<P, true, double>), dim3(blocks), dim3(256), 0, s,
                         (const double*)pos, n_total, offsets, (const float*)b.grid, g,
                         (double*)grad);
    else
      hipLaunchKernelGGL((k_gather_grad<P, false, double>), dim3(blocks), dim3(256), 0, s,
                         (const double*)pos, n_total, offsets, (const float*)b.grid, g,
                         (double*)grad);
  }
}

hipError_t launch_gather_grad(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                              int64_t n_total, const Buffers& b, void* grad, hipStream_t s) {
  switch (g.order) {
    case 1: dispatch_gather<1>(g, pos, dt, offsets, n_total, b, grad, s); break;
    case 2: dispatch_gather<2>(g, pos, dt, offsets, n_total, b, grad, s); break;
    case 3: dispatch_gather<3>(g, pos, dt, offsets, n_total, b, grad, s); break;
    default: dispatch_gather<4>(g, pos, dt, offsets, n_total, b, grad, s); break;
  }
  return hipGetLastError();
}

}  // namespace fsest
