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

__global__ void k_set_counts(const int64_t* offsets, int64_t n_total, int batch, int64_t* np,
                             double* norm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const int64_t c = offsets ? (offsets[i + 1] - offsets[i]) : n_total;
  np[i] = c;
  norm[2 * i] = (double)c;
  norm[2 * i + 1] = (double)c;
}

hipError_t launch_set_counts(const int64_t* offsets, int64_t n_total, int batch, int64_t* np,
                             double* norm, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counts, dim3((batch + 63) / 64), dim3(64), 0, s, offsets, n_total,
                     batch, np, norm);
  return hipGetLastError();
}

// ------------------------------------------------------------------ masses
// Per set, kWSlices workgroups each sum w and w^2 over a fixed slice of the
// set's particles (strided per thread, then a fixed tree over the
// workgroup), and a second pass adds the slices in order: the totals do not
// depend on scheduling.  The largest mass goes to stats[4] (non-negative
// floats order like their bit patterns) and any negative, NaN or infinite
// mass sets stats[5].
constexpr int kWThreads = 256;

__global__ __launch_bounds__(kWThreads) void k_weight_stats(const float* __restrict__ w,
                                                            const int64_t* __restrict__ offsets,
                                                            int64_t n_total,
                                                            double* __restrict__ wpart,
                                                            uint32_t* __restrict__ stats) {
  __shared__ double sa[kWThreads / 64], sb[kWThreads / 64];
  const int m = blockIdx.y, slice = blockIdx.x;
  const int64_t j0 = offsets ? offsets[m] : 0, j1 = offsets ? offsets[m + 1] : n_total;
  const int64_t len = j1 - j0;
  const int64_t s0 = j0 + len * slice / kWSlices, s1 = j0 + len * (slice + 1) / kWSlices;
  double a = 0.0, b = 0.0;
  float mx = 0.0f;
  bool bad = false;
  for (int64_t j = s0 + threadIdx.x; j < s1; j += kWThreads) {
    const float v = w[j];
    if (!(v >= 0.0f && v <= 3.402823466e38f)) {
      bad = true;
    } else {
      a += (double)v;
      b += (double)v * (double)v;
      if (v > mx) mx = v;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
    mx = fmaxf(mx, __shfl_down(mx, off, 64));
  }
  const unsigned long long anybad = __ballot(bad);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sa[wave] = a;
    sb[wave] = b;
    if (mx > 0.0f) atomicMax(&stats[4], __float_as_uint(mx));
    if (anybad) atomicOr(&stats[5], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < kWThreads / 64; ++i) {
      ta += sa[i];
      tb += sb[i];
    }
    double* dst = wpart + 2 * ((int64_t)m * kWSlices + slice);
    dst[0] = ta;
    dst[1] = tb;
  }
}

__global__ void k_weight_final(const double* __restrict__ wpart, int batch, double* __restrict__ norm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= batch) return;
  double ta = 0.0, tb = 0.0;
  for (int i = 0; i < kWSlices; ++i) {
    ta += wpart[2 * ((int64_t)m * kWSlices + i)];
    tb += wpart[2 * ((int64_t)m * kWSlices + i) + 1];
  }
  norm[2 * m] = ta;
  norm[2 * m + 1] = tb;
}

hipError_t launch_weight_stats(const float* w, const int64_t* offsets, int64_t n_total, int batch,
                               double* wpart, double* norm, uint32_t* stats, hipStream_t s) {
  hipError_t e = launch_fill_u32(stats + 4, 2, 0u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_weight_stats, dim3(kWSlices, batch), dim3(kWThreads), 0, s, w, offsets,
                     n_total, wpart, stats);
  hipLaunchKernelGGL(k_weight_final, dim3((batch + 63) / 64), dim3(64), 0, s, wpart, batch, norm);
  return hipGetLastError();
}

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

// ------------------------------------------------------------------ sort
// Bucket counts and each particle's rank inside its bucket.  A workgroup
// first counts its particles per bucket key in an LDS hash table (open
// addressing), then adds each distinct key's count to the global counter
// with one atomic, whose old value becomes the base of that key's ranks.
// Particles stored near each other in memory (simulation order) share
// buckets, so this removes most of the device-scope atomics.
constexpr int kCountThreads = 1024;
constexpr int kCountHash = 2048;  // slots, load factor <= 1/2
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

template <typename TP>
__global__ __launch_bounds__(kCountThreads) void k_bucket_count(
    const TP* __restrict__ pos, int64_t n_total, const int64_t* __restrict__ offsets, Geom g,
    uint32_t* __restrict__ counts, uint32_t* __restrict__ rank) {
  __shared__ uint32_t hkey[kCountHash];
  __shared__ uint32_t hval[kCountHash];
  for (int i = threadIdx.x; i < kCountHash; i += kCountThreads) {
    hkey[i] = kEmptyKey;
    hval[i] = 0u;
  }
  const int64_t j = (int64_t)blockIdx.x * kCountThreads + threadIdx.x;
  uint32_t key = kEmptyKey;
  if (j < n_total) {
    double x, y, z;
    load_pos(pos, j, x, y, z);
    const int mock = mock_of(offsets, g.batch, j);
    const int bx = base_cell(grid_coord(x, g.box, g.inv), g.n) / kBucket;
    const int by = base_cell(grid_coord(y, g.box, g.inv), g.n) / kBucket;
    const int bz = base_cell(grid_coord(z, g.box, g.inv), g.n) / kBucket;
    key = (uint32_t)(((int64_t)mock * g.nb + bx) * g.nb + by) * g.nb + bz;
  }
  __syncthreads();
  int slot = 0;
  uint32_t local = 0;
  if (key != kEmptyKey) {
    slot = (int)(key & (kCountHash - 1));
    while (true) {
      const uint32_t prev = atomicCAS(&hkey[slot], kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) break;
      slot = (slot + 1) & (kCountHash - 1);
    }
    local = atomicAdd(&hval[slot], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCountHash; i += kCountThreads) {
    const uint32_t k = hkey[i];
    if (k != kEmptyKey) hval[i] = atomicAdd(&counts[k], hval[i]);
  }
  __syncthreads();
  if (key != kEmptyKey) rank[j] = hval[slot] + local;
}

// Cell record of one particle, used by the deposit to decide which tiles a
// particle's stencils reach without redoing the float64 cell arithmetic:
// bits 16a .. 16a+15 hold the first-grid floor cell along axis a (floor(u)
// for even p, floor(u + 1/2) for odd p; mod N), bit 48 + a holds the step
// from it to the same floor on the grid shifted by H/2 (0 or 1).
// bits kRecFineShift.. carry a particle's bucket inside its super-bucket
// between the two passes of the two-level sort
constexpr int kRecFineShift = 52;

__device__ __forceinline__ uint64_t cell_record(double ux, double uy, double uz, const Geom& g) {
  const bool even = (g.order % 2) == 0;
  const double u[3] = {ux, uy, uz};
  uint64_t rec = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u2 = u[a] + 0.5;  // the interlaced grid's coordinate
    const double f1 = even ? floor(u[a]) : floor(u[a] + 0.5);
    const double f2 = even ? floor(u2) : floor(u2 + 0.5);
    const int c1 = (int)f1;  // in [0, N]
    rec |= (uint64_t)(c1 >= g.n ? c1 - g.n : c1) << (16 * a);
    rec |= (uint64_t)((int)(f2 - f1) & 1) << (48 + a);
  }
  return rec;
}

template <typename TP>
__global__ __launch_bounds__(256) void k_bucket_scatter(const TP* __restrict__ pos, int64_t n_total,
                                                        const int64_t* __restrict__ offsets, Geom g,
                                                        const uint32_t* __restrict__ boff,
                                                        const uint32_t* __restrict__ rank,
                                                        TP* __restrict__ sorted,
                                                        uint64_t* __restrict__ cells,
                                                        const float* __restrict__ w,
                                                        float* __restrict__ sw,
                                                        const uint32_t* __restrict__ stats) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_total) return;
  TP px = pos[3 * j + 0], py = pos[3 * j + 1], pz = pos[3 * j + 2];
  const int mock = mock_of(offsets, g.batch, j);
  const double ux = grid_coord((double)px, g.box, g.inv);
  const double uy = grid_coord((double)py, g.box, g.inv);
  const double uz = grid_coord((double)pz, g.box, g.inv);
  const int bx = base_cell(ux, g.n) / kBucket;
  const int by = base_cell(uy, g.n) / kBucket;
  const int bz = base_cell(uz, g.n) / kBucket;
  const uint32_t key = (uint32_t)(((int64_t)mock * g.nb + bx) * g.nb + by) * g.nb + bz;
  const int64_t dst = (int64_t)boff[key] + rank[j];
  sorted[3 * dst + 0] = px;
  sorted[3 * dst + 1] = py;
  sorted[3 * dst + 2] = pz;
  cells[dst] = cell_record(ux, uy, uz, g);
  if (w) sw[dst] = scaled_mass(w, j, stats);
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

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

static hipError_t scan_in_place(uint32_t* data, size_t n, uint32_t* tmp, uint32_t* maxcount,
                                hipStream_t s) {
  const int nblk = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_local, dim3(nblk), dim3(kScanThreads), 0, s, data, n, tmp, maxcount);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nblk);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk), dim3(kScanThreads), 0, s, data, n, tmp);
  return hipGetLastError();
}

// Counting sort with device-scope atomics: the general path, used when there
// are more super-buckets than one workgroup can histogram.
static hipError_t sort_atomic(const Geom& g, const void* pos, est_dtype dt,
                              const int64_t* offsets, int64_t n_total, const float* w,
                              const Buffers& b, hipStream_t s) {
  const size_t nkeys = (size_t)g.batch * g.nb * g.nb * g.nb;
  hipError_t e = launch_fill_u32(b.boff, nkeys + 1, 0u, s);
  if (e != hipSuccess) return e;
  const unsigned pblocks = (unsigned)((n_total + 255) / 256);
  const unsigned cblocks = (unsigned)((n_total + kCountThreads - 1) / kCountThreads);
  if (dt == EST_F32)
    hipLaunchKernelGGL(k_bucket_count<float>, dim3(cblocks), dim3(kCountThreads), 0, s,
                       (const float*)pos, n_total, offsets, g, b.boff, b.rank);
  else
    hipLaunchKernelGGL(k_bucket_count<double>, dim3(cblocks), dim3(kCountThreads), 0, s,
                       (const double*)pos, n_total, offsets, g, b.boff, b.rank);
  hipLaunchKernelGGL(k_copy_u32, dim3(2048), dim3(256), 0, s, b.boff, b.bcnt, nkeys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_in_place(b.boff, nkeys + 1, b.scan_tmp, b.stats, s)) != hipSuccess) return e;
  if (dt == EST_F32)
    hipLaunchKernelGGL(k_bucket_scatter<float>, dim3(pblocks), dim3(256), 0, s, (const float*)pos,
                       n_total, offsets, g, b.boff, b.rank, (float*)b.sorted, b.cells, w, b.sw,
                       b.stats);
  else
    hipLaunchKernelGGL(k_bucket_scatter<double>, dim3(pblocks), dim3(256), 0, s,
                       (const double*)pos, n_total, offsets, g, b.boff, b.rank,
                       (double*)b.sorted, b.cells, w, b.sw, b.stats);
  return hipGetLastError();
}

// ---- two-level sort without device-scope atomics
// Super-buckets are cubes of g.fb^3 buckets (g.nsup of them).  (A) each of
// nblk workgroups histograms a contiguous chunk of particles over the
// super-buckets in LDS; (B) the histograms, laid out super-major, are
// scanned, giving every (super-bucket, workgroup) pair its output offset;
// (C) each workgroup re-reads its chunk and moves every particle (position
// and cell record) into its super-bucket segment, ranking with LDS
// counters; (D) one workgroup per super-bucket counts its particles per
// bucket, writes the bucket offsets and counts, and moves the particles into
// bucket order.  Buckets are therefore contiguous in z inside a super-bucket;
// the deposit splits its bucket runs at super-bucket boundaries.
constexpr int kSortThreads = 1024;
constexpr int kSortBatch = 1;  // particles per thread handled together (loads in flight together)

__device__ __forceinline__ void particle_buckets(double ux, double uy, double uz, const Geom& g,
                                                 int& bx, int& by, int& bz) {
  bx = base_cell(ux, g.n) / kBucket;
  by = base_cell(uy, g.n) / kBucket;
  bz = base_cell(uz, g.n) / kBucket;
}

__device__ __forceinline__ int super_of(int mock, int bx, int by, int bz, const Geom& g) {
  return ((mock * g.sa + bx / g.fb) * g.sa + by / g.fb) * g.sa + bz / g.fb;
}

template <typename TP>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const TP* __restrict__ pos,
                                                            int64_t n_total,
                                                            const int64_t* __restrict__ offsets,
                                                            Geom g, int64_t chunk, int nblk,
                                                            uint32_t* __restrict__ hsup) {
  __shared__ uint32_t hist[kMaxSuper];
  for (int i = threadIdx.x; i < g.nsup; i += kSortThreads) hist[i] = 0u;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = (j0 + chunk < n_total) ? j0 + chunk : n_total;
  // kSortBatch particles per thread at a time, their loads issued together
  for (int64_t jb = j0 + threadIdx.x; jb < j1; jb += kSortBatch * kSortThreads) {
    double x[kSortBatch], y[kSortBatch], z[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const int64_t j = jb + (int64_t)q * kSortThreads;
      if (j < j1) load_pos(pos, j, x[q], y[q], z[q]);
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const int64_t j = jb + (int64_t)q * kSortThreads;
      if (j < j1) {
        int bx, by, bz;
        particle_buckets(grid_coord(x[q], g.box, g.inv), grid_coord(y[q], g.box, g.inv),
                         grid_coord(z[q], g.box, g.inv), g, bx, by, bz);
        atomicAdd(&hist[super_of(mock_of(offsets, g.batch, j), bx, by, bz, g)], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < g.nsup; i += kSortThreads)
    hsup[(int64_t)i * nblk + blockIdx.x] = hist[i];
}

template <typename TP>
__global__ __launch_bounds__(kSortThreads) void k_sort_super(
    const TP* __restrict__ pos, int64_t n_total, const int64_t* __restrict__ offsets, Geom g,
    int64_t chunk, int nblk, const uint32_t* __restrict__ hoff, TP* __restrict__ tpos,
    uint64_t* __restrict__ trec, const float* __restrict__ w, float* __restrict__ tw) {
  __shared__ uint32_t cur[kMaxSuper];
  for (int i = threadIdx.x; i < g.nsup; i += kSortThreads)
    cur[i] = hoff[(int64_t)i * nblk + blockIdx.x];
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = (j0 + chunk < n_total) ? j0 + chunk : n_total;
  for (int64_t jb = j0 + threadIdx.x; jb < j1; jb += kSortBatch * kSortThreads) {
    TP px[kSortBatch], py[kSortBatch], pz[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const int64_t j = jb + (int64_t)q * kSortThreads;
      if (j < j1) {
        px[q] = pos[3 * j + 0];
        py[q] = pos[3 * j + 1];
        pz[q] = pos[3 * j + 2];
      }
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const int64_t j = jb + (int64_t)q * kSortThreads;
      if (j < j1) {
        const double ux = grid_coord((double)px[q], g.box, g.inv);
        const double uy = grid_coord((double)py[q], g.box, g.inv);
        const double uz = grid_coord((double)pz[q], g.box, g.inv);
        int bx, by, bz;
        particle_buckets(ux, uy, uz, g, bx, by, bz);
        const int sup = super_of(mock_of(offsets, g.batch, j), bx, by, bz, g);
        const uint32_t fine = ((bx % g.fb) * g.fb + by % g.fb) * g.fb + bz % g.fb;
        const uint32_t p = atomicAdd(&cur[sup], 1u);
        tpos[3 * (int64_t)p + 0] = px[q];
        tpos[3 * (int64_t)p + 1] = py[q];
        tpos[3 * (int64_t)p + 2] = pz[q];
        trec[p] = cell_record(ux, uy, uz, g) | ((uint64_t)fine << kRecFineShift);
        if (w) tw[p] = w[j];
      }
    }
  }
}

template <typename TP>
__global__ __launch_bounds__(kSortThreads) void k_sort_fine(
    const TP* __restrict__ tpos, const uint64_t* __restrict__ trec, int64_t n_total, Geom g,
    int nblk, const uint32_t* __restrict__ hoff, TP* __restrict__ sorted,
    uint64_t* __restrict__ cells, uint32_t* __restrict__ boff, uint32_t* __restrict__ bcnt,
    uint32_t* __restrict__ stats, const float* __restrict__ tw, float* __restrict__ sw) {
  constexpr int kPer = kFineMax * kFineMax * kFineMax / kSortThreads;  // buckets per thread
  __shared__ uint32_t hist[kFineMax * kFineMax * kFineMax];
  __shared__ uint32_t wtot[kSortThreads / 64];
  const int sup = blockIdx.x;
  const int nf = g.fb * g.fb * g.fb;
  const uint32_t seg0 = hoff[(int64_t)sup * nblk];
  const uint32_t seg1 = (sup + 1 < g.nsup) ? hoff[(int64_t)(sup + 1) * nblk] : (uint32_t)n_total;
  for (int i = threadIdx.x; i < nf; i += kSortThreads) hist[i] = 0u;
  __syncthreads();
  for (uint32_t ib = seg0 + threadIdx.x; ib < seg1; ib += kSortBatch * kSortThreads) {
    uint64_t r[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const uint32_t i = ib + q * kSortThreads;
      r[q] = (i < seg1) ? trec[i] : 0ull;
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q)
      if (ib + q * kSortThreads < seg1) atomicAdd(&hist[(uint32_t)(r[q] >> kRecFineShift)], 1u);
  }
  __syncthreads();
  // exclusive scan of hist[0, nf): kPer consecutive buckets per thread
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint32_t c[kPer], run = 0, mx = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int f = t * kPer + q;
    c[q] = (f < nf) ? hist[f] : 0u;
    mx = max(mx, c[q]);
    run += c[q];
  }
  uint32_t incl = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wtot[wave] = incl;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_down((int)mx, o, 64));
  if (lane == 0) atomicMax(&stats[0], mx);
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wtot[w];
  uint32_t start = seg0 + before + incl - run;
  // bucket offsets and counts, in global key order
  const int ms = sup / (g.sa * g.sa * g.sa), srem = sup % (g.sa * g.sa * g.sa);
  const int sx = srem / (g.sa * g.sa), sy = (srem / g.sa) % g.sa, sz = srem % g.sa;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int f = t * kPer + q;
    if (f < nf) {
      const int fx = f / (g.fb * g.fb), fy = (f / g.fb) % g.fb, fz = f % g.fb;
      const int64_t key = (((int64_t)ms * g.nb + sx * g.fb + fx) * g.nb + sy * g.fb + fy) * g.nb +
                          sz * g.fb + fz;
      boff[key] = start;
      bcnt[key] = c[q];
      hist[f] = start - seg0;
    }
    start += c[q];
  }
  __syncthreads();
  for (uint32_t ib = seg0 + threadIdx.x; ib < seg1; ib += kSortBatch * kSortThreads) {
    uint64_t r[kSortBatch];
    TP px[kSortBatch], py[kSortBatch], pz[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const uint32_t i = ib + q * kSortThreads;
      if (i < seg1) {
        r[q] = trec[i];
        px[q] = tpos[3 * (int64_t)i + 0];
        py[q] = tpos[3 * (int64_t)i + 1];
        pz[q] = tpos[3 * (int64_t)i + 2];
      }
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      if (ib + q * kSortThreads < seg1) {
        const uint32_t p = seg0 + atomicAdd(&hist[(uint32_t)(r[q] >> kRecFineShift)], 1u);
        sorted[3 * (int64_t)p + 0] = px[q];
        sorted[3 * (int64_t)p + 1] = py[q];
        sorted[3 * (int64_t)p + 2] = pz[q];
        cells[p] = r[q] & ((1ull << kRecFineShift) - 1ull);
        if (tw) sw[p] = scaled_mass(tw, ib + q * kSortThreads, stats);
      }
    }
  }
}

template <typename TP>
static hipError_t sort_two_level(const Geom& g, const TP* pos, const int64_t* offsets,
                                 int64_t n_total, const float* w, const Buffers& b, hipStream_t s) {
  int nblk = (int)((n_total + 4095) / 4096);
  if (nblk > kMaxSortBlocks) nblk = kMaxSortBlocks;
  const int64_t chunk = (n_total + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_sort_hist<TP>, dim3(nblk), dim3(kSortThreads), 0, s, pos, n_total,
                     offsets, g, chunk, nblk, b.hsup);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the scan's largest-entry output is not a bucket count here
  if ((e = scan_in_place(b.hsup, (size_t)g.nsup * nblk, b.scan_tmp, b.stats + 2, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_sort_super<TP>, dim3(nblk), dim3(kSortThreads), 0, s, pos, n_total,
                     offsets, g, chunk, nblk, b.hsup, (TP*)b.tpos, b.trec, w, b.tw);
  hipLaunchKernelGGL(k_sort_fine<TP>, dim3(g.nsup), dim3(kSortThreads), 0, s, (const TP*)b.tpos,
                     b.trec, n_total, g, nblk, b.hsup, (TP*)b.sorted, b.cells, b.boff, b.bcnt,
                     b.stats, w ? b.tw : nullptr, b.sw);
  return hipGetLastError();
}

hipError_t launch_sort(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                       int64_t n_total, const float* w, const Buffers& b, hipStream_t s) {
  hipError_t e = launch_fill_u32(b.stats, 4, 0u, s);
  if (e != hipSuccess) return e;
  if (g.nsup > kMaxSuper) return sort_atomic(g, pos, dt, offsets, n_total, w, b, s);
  if (dt == EST_F32) return sort_two_level(g, (const float*)pos, offsets, n_total, w, b, s);
  return sort_two_level(g, (const double*)pos, offsets, n_total, w, b, s);
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

// ------------------------------------------------------------------ deposit
// Fixed-point accumulation.  LDS float atomics are ~20x slower than integer
// ones on gfx950, so a workgroup sums its tile in unsigned integers: a weight
// product w in [0, 1] adds floor(w * S + 1/2).  Two formats:
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

// The base cells of the particles that reach one cell span p + 1 cells per
// axis (both grids), so they meet at most 2 buckets per axis for p <= 4 and
// 3 for p = 5, 6.
template <int P>
__device__ __forceinline__ int narrow_bits(uint32_t maxcount) {
  const double bound = (P <= 4 ? 8.0 : 27.0) * (double)(maxcount > 0 ? maxcount : 1);
  int f = 0;
  while (f < 31 && bound * (ldexp(1.0, f + 1) + 1.0) < 4294967295.0) ++f;
  return f;
}

// LDS layout of a deposit workgroup, in 32-bit words:
//   [0, kItemCap)            particle index of each work item
//   [.., + kItemCap/4)       item meta bytes: bank class (6 bits) | grid << 6
//   [.., + kItemCap/2)       item order after sorting by bank class (u16)
//   [kAccWord, ...)          tile accumulators, one region of kGridWords
//                            elements per grid
// Each tile row holds h = zhalo<p>() extra cells on both z sides (3 up to
// p = 4, p - 1 above), so every cell of a stencil row that reaches the tile
// has an address: a stencil is added at base + i*kPlane + k*kRow + l with
// compile-time offsets, rows outside the tile in x or y are skipped, and
// halo cells are dropped (or, when the tile is the whole periodic grid,
// folded back) at write-out.  kRow and kPlane make the 64 offsets
// i*kPlane + k*kRow + l (i, k, l < 4) distinct mod 64, so for p <= 4 two
// stencils whose bases differ mod 64 never share an LDS bank in one
// instruction; work items are ordered by that residue ("bank class") and
// each wave takes items spread evenly over the order, which keeps the
// classes of its 64 lanes distinct except where a class holds more items
// than there are waves in the flush.
constexpr int kZHalo = 3;  // orders up to 4; zhalo<P>() in general
constexpr int kMaxOrder = 6;
template <int P>
__device__ __host__ constexpr int zhalo() { return P <= 4 ? kZHalo : P - 1; }
constexpr int kRow = 28;
constexpr int kPlane = 464;
constexpr int kGridWords = kTileMax * kPlane;
constexpr int kItemCap = 2048;
constexpr int kAccWord = kItemCap + kItemCap / 4 + kItemCap / 2;

constexpr bool offsets_cover_banks() {
  bool seen[64] = {};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) {
        const int r = (i * kPlane + k * kRow + l) % 64;
        if (seen[r]) return false;
        seen[r] = true;
      }
  return true;
}
static_assert(offsets_cover_banks(), "stencil offsets must cover the 64 banks");
static_assert(kRow >= kTileMax + 2 * (kMaxOrder - 1) && kPlane >= kTileMax * kRow, "tile pitches");
static_assert(kAccWord % 64 == 0 && kGridWords % 64 == 0, "regions start on bank 0");
// the lowest element a stencil base can address lies kAccMargin below a region
constexpr int kAccMargin = (kMaxOrder - 1) * (kPlane + kRow);
// 64-bit accumulators start further in, so that their margin also fits
constexpr int kAccWordWide = 5120;
static_assert(kAccWord >= kAccMargin && kAccWordWide / 2 >= kAccMargin && kAccWordWide % 64 == 0,
              "base addresses stay non-negative");
template <typename AT>
__device__ __host__ constexpr int acc_first_word() { return sizeof(AT) == 4 ? kAccWord : kAccWordWide; }

struct DepRanges {
  uint32_t start[72];
  uint32_t pref[73];
  int count;
};

// First cell of the p-point stencil along one axis (not wrapped) and its
// weights times `scale`, for grid coordinate u (the cell choice of
// stencil_1d, whose weights these are).
template <int P>
__device__ __forceinline__ int stencil_first(double u, float scale, float (&w)[P]) {
  int cell[P];
  stencil_1d<P>(u, 1 << 30, cell, w);
  const double fl = (P % 2 == 0) ? floor(u) : floor(u + 0.5);
#pragma unroll
  for (int i = 0; i < P; ++i) w[i] *= scale;
  return (int)fl - ((P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2);
}

template <int P>
__device__ __forceinline__ int first_cell(double u) {
  const double fl = (P % 2 == 0) ? floor(u) : floor(u + 0.5);
  return (int)fl - ((P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2);
}

// Position of a stencil's first cell relative to the tile origin t0, mod N.
// For a tile smaller than the grid the result lies in [-(P-1), n - P + 1)
// and the stencil reaches the tile's LDS block iff it is < kTileMax (which
// needs N >= kTileMax + P - 1); for a tile that is the whole grid (t0 = 0)
// it lies in [0, n).  `first` is a record cell (in [0, N)) minus the stencil
// offset plus the interlacing step, so first - t0 lies in [-(P-1) - N + 1, N].
// WRAP: kPeriodic (the tile is the whole grid), kMasked (tile smaller than a
// power-of-two grid: the residue is a mask), kGeneral (any other N).
constexpr int kPeriodic = 0, kMasked = 1, kGeneral = 2;

template <int P, int WRAP>
__device__ __forceinline__ int rel_first(int first, int t0, int n) {
  int r = first - t0;
  if constexpr (WRAP == kPeriodic) {
    r = r < 0 ? r + n : r;
    return r >= n ? r - n : r;
  } else if constexpr (WRAP == kMasked) {
    r &= n - 1;
    return (r >= n - (P - 1)) ? r - n : r;
  } else {
    r = r < -(P - 1) ? r + n : r;
    return (r >= n - (P - 1)) ? r - n : r;
  }
}

template <int P, int WRAP>
__device__ __forceinline__ bool reaches_tile(int rx, int ry, int rz) {
  if constexpr (WRAP == kPeriodic) return true;
  else return rx < kTileMax && ry < kTileMax && rz < kTileMax;
}

template <int P>
__device__ __forceinline__ int bank_class(int rx, int ry, int rz) {
  return (rx * kPlane + ry * kRow + rz + zhalo<P>()) & 63;
}

// Adds one grid's footprint of one particle to the tile.
template <int P, typename AT, int WRAP>
__device__ __forceinline__ void deposit_item(double x, double y, double z, int gi, const Geom& g,
                                             int t0x, int t0y, int t0z, AT* sm, float scale,
                                             int mk) {
  const int n = g.n;
  // grid gi is sampled at u + 1/2 on the axes whose bit is set in its mask mk
  float wx[P], wy[P], wz[P];
  const int fx = stencil_first<P>(grid_coord(x, g.box, g.inv) + ((mk & 1) ? 0.5 : 0.0), scale, wx);
  const int fy = stencil_first<P>(grid_coord(y, g.box, g.inv) + ((mk & 2) ? 0.5 : 0.0), 1.0f, wy);
  const int fz = stencil_first<P>(grid_coord(z, g.box, g.inv) + ((mk & 4) ? 0.5 : 0.0), 1.0f, wz);
  constexpr bool PERIODIC = WRAP == kPeriodic;
  const int rx = rel_first<P, WRAP>(fx, t0x, n);
  const int ry = rel_first<P, WRAP>(fy, t0y, n);
  const int rz = rel_first<P, WRAP>(fz, t0z, n);
  const int region = (acc_first_word<AT>() * 4 / (int)sizeof(AT)) + gi * kGridWords;
  if constexpr (PERIODIC) {
    // the tile is the whole grid (n <= kTileMax): x and y wrap, z runs into
    // the upper halo and is folded back at write-out
    AT* zrow = sm + region + rz + zhalo<P>();
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int xo = (rx + i >= n ? rx + i - n : rx + i) * kPlane;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        AT* row = zrow + xo + (ry + k >= n ? ry + k - n : ry + k) * kRow;
        const float wxy = wx[i] * wy[k];
#pragma unroll
        for (int l = 0; l < P; ++l)
          atomicAdd(&row[l], (AT)(uint32_t)__builtin_fmaf(wxy, wz[l], 0.5f));
      }
    }
  } else {
    AT* base = sm + region + rx * kPlane + ry * kRow + rz + zhalo<P>();
#pragma unroll
    for (int i = 0; i < P; ++i) {
      if ((unsigned)(rx + i) >= (unsigned)kTileMax) continue;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if ((unsigned)(ry + k) >= (unsigned)kTileMax) continue;
        const float wxy = wx[i] * wy[k];
#pragma unroll
        for (int l = 0; l < P; ++l)
          atomicAdd(&base[i * kPlane + k * kRow + l],
                    (AT)(uint32_t)__builtin_fmaf(wxy, wz[l], 0.5f));
      }
    }
  }
}

// Segment of each lane's candidate: a scalar search for the wave's first
// item c0, then the few segment starts inside the wave's 64 items.
__device__ __forceinline__ int find_segment(const DepRanges& rg, int nr, uint32_t c0,
                                            uint32_t item) {
  int lo = 0, hi = nr;  // pref[lo] <= c0 < pref[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((uint32_t)__builtin_amdgcn_readfirstlane((int)rg.pref[mid]) <= c0) lo = mid;
    else hi = mid;
  }
  int seg = lo;
  for (int t = lo + 1; t < nr; ++t) {
    const uint32_t pt = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.pref[t]);
    if (pt > c0 + 63) break;
    if (item >= pt) seg = t;
  }
  return seg;
}

// One workgroup owns one T^3 output tile (T = min(kTileMax, N)) of every
// grid at a time.  Per tile: (1) the particles of the buckets that can
// reach the tile are scanned in rounds of blockDim items; each grid whose
// stencil reaches the tile becomes a work item in an LDS list and counts
// towards its bank class; (2) whenever the list might overflow, it is
// counting-sorted by class and deposited with LDS integer atomics, lane l of
// virtual wave r taking sorted item r + l * W (W = virtual waves in the
// flush); (3) the finished tile is scaled back to float and written once.
// `dynamic`: tiles are taken from a global counter (stats[1], zeroed with
// the sort) instead of one tile per workgroup.  `xcd`: consecutive tiles go
// to the same XCD (workgroup b runs on XCD b mod 8), so the buckets that
// neighbouring tiles share are read through one L2.
// WT: per-particle masses (sw, bucket order, divided by the largest mass);
// a separate instantiation so that the equal-mass kernel keeps its registers
// IL: 0 one grid; 1 the interlaced pair (masks 0 and 7); 2 a pair of grids
// with run-time masks (mask_a, mask_b) written to slab q of each set
template <int P, int IL, typename TP, bool WIDE, int WRAP, bool WT>
__global__ __launch_bounds__(1024) void k_deposit(const TP* __restrict__ sorted,
                                                  const uint64_t* __restrict__ cells,
                                                  const uint32_t* __restrict__ boff,
                                                  const uint32_t* __restrict__ bcnt, float* grid,
                                                  Geom g, uint32_t* __restrict__ stats,
                                                  int exclusive, int dynamic, int xcd,
                                                  const float* __restrict__ sw, int q, int mask_a,
                                                  int mask_b) {
  using AT = typename std::conditional<WIDE, unsigned long long, unsigned>::type;
  constexpr int NG = IL ? 2 : 1;
  constexpr int MAXW = 16;  // waves per workgroup (1024 threads)
  constexpr int kWords = acc_first_word<AT>() + NG * kGridWords * (int)(sizeof(AT) / 4);
  __shared__ __align__(16) uint32_t smem[kWords];
  __shared__ DepRanges rg;
  __shared__ int wave_cnt[MAXW];
  __shared__ int cls_cnt[64];
  __shared__ int cls_cur[64];
  __shared__ int fill, next_tile;
  uint32_t* item_j = smem;
  uint8_t* item_meta = reinterpret_cast<uint8_t*>(smem + kItemCap);
  uint16_t* item_order = reinterpret_cast<uint16_t*>(smem + kItemCap + kItemCap / 4);
  AT* sm = reinterpret_cast<AT*>(smem);
  const int acc0 = acc_first_word<AT>() * 4 / (int)sizeof(AT);

  // fixed-point format for this deposit (uniform over the grid)
  const int nbits = narrow_bits<P>(stats[0]);
  if (!WIDE && nbits < kNarrowMinBits) return;                // the wide kernel does it
  if (WIDE && !exclusive && nbits >= kNarrowMinBits) return;  // the narrow one does it
  const float scale = WIDE ? kFixWide : ldexpf(1.0f, nbits);
  const double inv_scale = 1.0 / (double)scale;
  // masses: items carry w / w_max (in [0, 1], so the bounds above hold) and
  // the tile is multiplied back by w_max; an invalid mass makes it NaN
  float wmul = 1.0f;
  if constexpr (WT) wmul = stats[5] ? __builtin_nanf("") : __uint_as_float(stats[4]);

  const int n = g.n, T = g.tile, nb = g.nb;
  const int tpa = (n + T - 1) / T;  // tiles per axis; the last one is ragged when T does not divide N
  const int64_t tiles_per_set = (int64_t)tpa * tpa * tpa;
  const int64_t ntiles = (int64_t)g.batch * tiles_per_set;
  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (nthreads + 63) >> 6;
  const bool remap = xcd && !dynamic && (int64_t)gridDim.x == ntiles && (ntiles & 7) == 0;

  int64_t b = blockIdx.x;
  if (dynamic) {
    if (threadIdx.x == 0) next_tile = (int)atomicAdd(&stats[1], 1u);
    __syncthreads();
    b = next_tile;
  }
  while (b < ntiles) {
    const int64_t tid_all = remap ? ((b & 7) * (ntiles >> 3) + (b >> 3)) : b;
    const int mock = (int)(tid_all / tiles_per_set);
    const int trem = (int)(tid_all % tiles_per_set);
    const int tx = trem / (tpa * tpa), ty = (trem / tpa) % tpa, tz = trem % tpa;
    const int t0x = tx * T, t0y = ty * T, t0z = tz * T;
    // cells of this tile per axis (a multiple of kBucket)
    const int ex = min(T, n - t0x), ey = min(T, n - t0y), ez = min(T, n - t0z);

    if (threadIdx.x < 64) cls_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) fill = 0;

    // bucket neighbourhood: buckets of cells t0-3 .. t0+T, or every bucket
    int cnt = T / kBucket + 2;
    if (cnt > nb) cnt = nb;
    const int b0x = (cnt == nb) ? 0 : (t0x / kBucket - 1 + nb) % nb;
    const int b0y = (cnt == nb) ? 0 : (t0y / kBucket - 1 + nb) % nb;
    const int b0z = (cnt == nb) ? 0 : (t0z / kBucket - 1 + nb) % nb;
    const int ncomb = cnt * cnt;  // <= 36
    const int64_t mbase = (int64_t)mock * nb * nb * nb;
    if (wave == 0) {
      // a column's run of cnt buckets in z is contiguous in memory except
      // where it crosses a super-bucket edge (every g.fb buckets, which
      // includes the periodic wrap): at most two pieces
      uint32_t s0 = 0, e0 = 0, s1 = 0, e1 = 0;
      if (lane < ncomb) {
        const int ix = lane / cnt, iy = lane % cnt;
        const int bx = (b0x + ix) % nb, by = (b0y + iy) % nb;
        const int64_t row = mbase + ((int64_t)bx * nb + by) * nb;
        const int z1 = b0z + cnt;                       // exclusive end, may pass nb
        const int zs = (b0z / g.fb + 1) * g.fb;         // next super-bucket edge
        const int za = z1 < zs ? z1 : zs;               // end of the first piece
        s0 = boff[row + b0z];
        e0 = boff[row + za - 1] + bcnt[row + za - 1];
        if (z1 > zs) {
          const int zb = zs % nb, ze = zb + (z1 - zs);
          s1 = boff[row + zb];
          e1 = boff[row + ze - 1] + bcnt[row + ze - 1];
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
    // the other waves clear the tile while wave 0 waits for the offsets
    {
      uint4* z4 = reinterpret_cast<uint4*>(smem + acc_first_word<AT>());
      constexpr int kZero4 = (kWords - acc_first_word<AT>()) / 4;
      for (int i = threadIdx.x; i < kZero4; i += nthreads) z4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const uint32_t total = rg.pref[rg.count];
    const int nr = rg.count;

    // rounds of blockDim candidates; the cell records of kPre rounds are
    // loaded together so that their latencies overlap
    constexpr int kPre = 4;
    constexpr int off = (P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2;
    for (uint32_t rb = 0; rb < total; rb += kPre * nthreads) {
      uint32_t jj[kPre];
      uint64_t rec[kPre];
#pragma unroll
      for (int q = 0; q < kPre; ++q) {
        const uint32_t r0 = rb + q * nthreads;
        const uint32_t item = r0 + threadIdx.x;
        jj[q] = 0;
        rec[q] = 0;
        if (r0 < total) {
          const int seg = find_segment(rg, nr, r0 + (uint32_t)(wave * 64), item);
          if (item < total) {
            jj[q] = rg.start[seg] + (item - rg.pref[seg]);
            rec[q] = cells[jj[q]];
          }
        }
      }
#pragma unroll 1
      for (int q = 0; q < kPre; ++q) {
        const uint32_t r0 = rb + q * nthreads;
        if (r0 >= total) break;
        // (1) candidates of this round -> work items
        const uint32_t item = r0 + threadIdx.x;
        const uint32_t j = jj[0];
        bool ok[NG];
        int cls[NG];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          ok[gi] = false;
          cls[gi] = 0;
        }
        if (item < total) {
          const uint64_t r = rec[0];
          const int cx = (int)(r & 0xFFFF) - off;
          const int cy = (int)((r >> 16) & 0xFFFF) - off;
          const int cz = (int)((r >> 32) & 0xFFFF) - off;
#pragma unroll
          for (int gi = 0; gi < NG; ++gi) {
            const int mk = (IL == 2) ? (gi ? mask_b : mask_a) : (gi ? 7 : 0);
            const int sx = (mk & 1) ? (int)((r >> 48) & 1) : 0;
            const int sy = (mk & 2) ? (int)((r >> 49) & 1) : 0;
            const int sz = (mk & 4) ? (int)((r >> 50) & 1) : 0;
            const int rx = rel_first<P, WRAP>(cx + sx, t0x, n);
            const int ry = rel_first<P, WRAP>(cy + sy, t0y, n);
            const int rz = rel_first<P, WRAP>(cz + sz, t0z, n);
            ok[gi] = reaches_tile<P, WRAP>(rx, ry, rz);
            cls[gi] = bank_class<P>(rx, ry, rz);
          }
        }
#pragma unroll
        for (int t = 0; t + 1 < kPre; ++t) {
          jj[t] = jj[t + 1];
          rec[t] = rec[t + 1];
        }
        unsigned long long bal[NG];
        int mine = 0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          bal[gi] = __ballot(ok[gi]);
          mine += __popcll(bal[gi]);
        }
        if (lane == 0) wave_cnt[wave] = mine;
        __syncthreads();
        int before = 0, tot = 0;
        for (int w = 0; w < nwaves; ++w) {
          const int c = wave_cnt[w];
          before += (w < wave) ? c : 0;
          tot += c;
        }
        const int f0 = fill;
        const unsigned long long below = (1ull << lane) - 1ull;
        int pos = f0 + before;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          if (ok[gi]) {
            const int p = pos + __popcll(bal[gi] & below);
            item_j[p] = j;
            item_meta[p] = (uint8_t)(cls[gi] | (gi << 6));
            atomicAdd(&cls_cnt[cls[gi]], 1);
          }
          pos += __popcll(bal[gi]);
        }
        __syncthreads();
        const int m = f0 + tot;
        const bool last = r0 + nthreads >= total;
        if (m + NG * nthreads > kItemCap || last) {
          // (2) sort the items by bank class, then deposit them
          if (wave == 0) {
            const int c = cls_cnt[lane];
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
              const int t = __shfl_up(incl, o, 64);
              if (lane >= o) incl += t;
            }
            cls_cur[lane] = incl - c;
            cls_cnt[lane] = 0;
          }
          __syncthreads();
          for (int e = threadIdx.x; e < m; e += nthreads)
            item_order[atomicAdd(&cls_cur[item_meta[e] & 63], 1)] = (uint16_t)e;
          __syncthreads();
          // lane l of virtual wave r takes item r + l W; each item's position
          // is loaded one iteration ahead
          const int W = (m + 63) >> 6;
          const int vend = 64 * W;
          int e_cur = -1;
          TP px = 0, py = 0, pz = 0;
          {
            const int v = threadIdx.x;
            const int p = (v >> 6) + (v & 63) * W;
            if (v < vend && p < m) {
              e_cur = item_order[p];
              const int64_t jq = item_j[e_cur];
              px = sorted[3 * jq + 0];
              py = sorted[3 * jq + 1];
              pz = sorted[3 * jq + 2];
            }
          }
          for (int v = threadIdx.x; v < vend; v += nthreads) {
            const int vn = v + nthreads;
            const int pn = (vn >> 6) + (vn & 63) * W;
            int e_nxt = -1;
            TP nx = 0, ny = 0, nz = 0;
            if (vn < vend && pn < m) {
              e_nxt = item_order[pn];
              const int64_t jq = item_j[e_nxt];
              nx = sorted[3 * jq + 0];
              ny = sorted[3 * jq + 1];
              nz = sorted[3 * jq + 2];
            }
            if (e_cur >= 0) {
              float sc = scale;
              if constexpr (WT) sc *= sw[item_j[e_cur]];
              const int gi = item_meta[e_cur] >> 6;
              const int mk = (IL == 2) ? (gi ? mask_b : mask_a) : (gi ? 7 : 0);
              deposit_item<P, AT, WRAP>((double)px, (double)py, (double)pz, gi, g, t0x, t0y, t0z,
                                        sm, sc, mk);
            }
            e_cur = e_nxt;
            px = nx;
            py = ny;
            pz = nz;
          }
          __syncthreads();
          if (threadIdx.x == 0) fill = 0;
        } else if (threadIdx.x == 0) {
          fill = m;
        }
        __syncthreads();
      }
    }

    // (3) write the tile (halo cells dropped, or folded back when periodic)
    const int slab = (IL == 2) ? mock * g.npair + q : mock;
    if constexpr (WRAP != kPeriodic) {
      // four consecutive z cells per thread; the narrow scale is a power of
      // two, so float(sum) * 2^-F rounds exactly like the double product
      constexpr int TT = kTileMax;
      const float inv_f = (float)inv_scale;
      for (int i = threadIdx.x; i < TT * TT * TT / 4; i += nthreads) {
        const int lx = i / (TT * TT / 4), ly = (i / (TT / 4)) % TT, lz = (i % (TT / 4)) * 4;
        if (lx >= ex || ly >= ey || lz >= ez) continue;  // outside a ragged tile
        float v[NG][4];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          const int a = acc0 + gi * kGridWords + lx * kPlane + ly * kRow + lz + zhalo<P>();
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const AT s = sm[a + q];
            v[gi][q] = (WIDE ? (float)((double)s * inv_scale) : (float)s * inv_f) * wmul;
          }
        }
        if constexpr (IL) {
          float4* dst = reinterpret_cast<float4*>(
              reinterpret_cast<float2*>(grid) + complex_index(g, slab, t0x + lx, t0y + ly, t0z + lz));
          dst[0] = make_float4(v[0][0], v[NG - 1][0], v[0][1], v[NG - 1][1]);
          dst[1] = make_float4(v[0][2], v[NG - 1][2], v[0][3], v[NG - 1][3]);
        } else {
          *reinterpret_cast<float4*>(grid + real_cell_index(g, slab, t0x + lx, t0y + ly, t0z + lz)) =
              make_float4(v[0][0], v[0][1], v[0][2], v[0][3]);
        }
      }
    } else {
      for (int i = threadIdx.x; i < T * T * T; i += nthreads) {
        const int lx = i / (T * T), ly = (i / T) % T, lz = i % T;
        float v[NG];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          const int a = acc0 + gi * kGridWords + lx * kPlane + ly * kRow + lz + zhalo<P>();
          AT s = sm[a];
          if (lz < zhalo<P>()) s += sm[a + T];
          v[gi] = (float)((double)s * inv_scale) * wmul;
        }
        if constexpr (IL) {
          reinterpret_cast<float2*>(grid)[complex_index(g, slab, t0x + lx, t0y + ly, t0z + lz)] =
              make_float2(v[0], v[NG - 1]);
        } else {
          grid[real_cell_index(g, slab, t0x + lx, t0y + ly, t0z + lz)] = v[0];
        }
      }
    }
    if (dynamic) {
      __syncthreads();  // every thread has read next_tile and finished the tile
      if (threadIdx.x == 0) next_tile = (int)atomicAdd(&stats[1], 1u);
      __syncthreads();
      b = next_tile;
    } else {
      b += gridDim.x;
      __syncthreads();
    }
  }
}

template <int P, int IL, typename TP, int WRAP, bool WT>
static void deposit_launch(const Geom& g, const Buffers& b, int threads, bool narrow, bool xcd,
                           const float* sw, int q, int ma, int mb, hipStream_t s) {
  const int tpa = (g.n + g.tile - 1) / g.tile;
  const int64_t ntiles = (int64_t)g.batch * tpa * tpa * tpa;
  if (narrow)
    hipLaunchKernelGGL((k_deposit<P, IL, TP, false, WRAP, WT>), dim3((unsigned)ntiles), dim3(threads),
                       0, s, (const TP*)b.sorted, b.cells, b.boff, b.bcnt, (float*)b.grid, g, b.stats, 0,
                       0, xcd ? 1 : 0, sw, q, ma, mb);
  // the 64-bit kernel holds one workgroup per CU; it takes tiles from a
  // counter, so when the 32-bit kernel does the work it costs one short wave
  // per workgroup
  const unsigned wblocks = (unsigned)(ntiles < 1024 ? ntiles : 1024);
  hipLaunchKernelGGL((k_deposit<P, IL, TP, true, WRAP, WT>), dim3(wblocks), dim3(threads), 0, s,
                     (const TP*)b.sorted, b.cells, b.boff, b.bcnt, (float*)b.grid, g, b.stats,
                     narrow ? 0 : 1, 1, 0, sw, q, ma, mb);
}

template <int P, int IL, int WRAP>
static void dispatch_deposit_w(const Geom& g, est_dtype dt, const Buffers& b, int threads,
                               bool narrow, bool xcd, const float* sw, int q, int ma, int mb,
                               hipStream_t s) {
  if (sw) {
    if (dt == EST_F32) deposit_launch<P, IL, float, WRAP, true>(g, b, threads, narrow, xcd, sw, q, ma, mb, s);
    else deposit_launch<P, IL, double, WRAP, true>(g, b, threads, narrow, xcd, sw, q, ma, mb, s);
  } else {
    if (dt == EST_F32) deposit_launch<P, IL, float, WRAP, false>(g, b, threads, narrow, xcd, nullptr, q, ma, mb, s);
    else deposit_launch<P, IL, double, WRAP, false>(g, b, threads, narrow, xcd, nullptr, q, ma, mb, s);
  }
}

template <int P, int IL>
static void dispatch_deposit_t(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                               int threads, const float* sw, int q, int ma, int mb, hipStream_t s) {
  const bool narrow = tu.dep_narrow != 0;
  const bool xcd = tu.dep_xcd != 0;
  if (g.tile == g.n)
    dispatch_deposit_w<P, IL, kPeriodic>(g, dt, b, threads, narrow, xcd, sw, q, ma, mb, s);
  else if ((g.n & (g.n - 1)) == 0)
    dispatch_deposit_w<P, IL, kMasked>(g, dt, b, threads, narrow, xcd, sw, q, ma, mb, s);
  else
    dispatch_deposit_w<P, IL, kGeneral>(g, dt, b, threads, narrow, xcd, sw, q, ma, mb, s);
}

template <int P>
static void dispatch_deposit_p(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                               int threads, const float* sw, hipStream_t s) {
  if (g.code == 0) {
    dispatch_deposit_t<P, 0>(g, dt, b, tu, threads, sw, 0, 0, 0, s);
  } else if (g.code == 1) {
    dispatch_deposit_t<P, 1>(g, dt, b, tu, threads, sw, 0, 0, 7, s);
  } else {
    // one pass per slab; the 64-bit kernel's tile counter restarts each time
    for (int q = 0; q < g.npair; ++q) {
      if (q > 0) launch_fill_u32(b.stats + 1, 1, 0u, s);
      dispatch_deposit_t<P, 2>(g, dt, b, tu, threads, sw, q, grid_mask(g.code, 2 * q),
                               grid_mask(g.code, 2 * q + 1), s);
    }
  }
}

hipError_t launch_deposit(const Geom& g, est_dtype dt, const Buffers& b, const Tune& tu,
                          bool weighted, hipStream_t s) {
  int threads = tu.dep_threads;
  if (threads != 256 && threads != 512 && threads != 1024) threads = 1024;
  const float* sw = weighted ? b.sw : nullptr;
  switch (g.order) {
    case 1: dispatch_deposit_p<1>(g, dt, b, tu, threads, sw, s); break;
    case 2: dispatch_deposit_p<2>(g, dt, b, tu, threads, sw, s); break;
    case 3: dispatch_deposit_p<3>(g, dt, b, tu, threads, sw, s); break;
    case 4: dispatch_deposit_p<4>(g, dt, b, tu, threads, sw, s); break;
    case 5: dispatch_deposit_p<5>(g, dt, b, tu, threads, sw, s); break;
    default: dispatch_deposit_p<6>(g, dt, b, tu, threads, sw, s); break;
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
    // grid `which` (1-based) is component (which - 1) % 2 of slab (which - 1) / 2
    const int slab = mock * g.npair + (which - 1) / 2;
    if (g.il)
      dst[i] = grid[2 * complex_index(g, slab, x, y, z) + ((which - 1) & 1)];
    else
      dst[i] = grid[real_cell_index(g, slab, x, y, z)];
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
                                                     const float* __restrict__ w,
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
  // a particle of mass w_j deposits w_j times the kernel
  const double sc = -(double)n / g.box * (w ? (double)w[j] : 1.0);
  grad[3 * j + 0] = (TP)(sc * gx);
  grad[3 * j + 1] = (TP)(sc * gy);
  grad[3 * j + 2] = (TP)(sc * gz);
}

template <int P>
static void dispatch_gather(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                            int64_t n_total, const float* w, const Buffers& b, void* grad,
                            hipStream_t s) {
  const unsigned blocks = (unsigned)((n_total + 255) / 256);
  if (dt == EST_F32) {
    if (g.il)
      hipLaunchKernelGGL((k_gather_grad<P, true, float>), dim3(blocks), dim3(256), 0, s,
                         (const float*)pos, n_total, offsets, (const float*)b.grid, g, w, (float*)grad);
    else
      hipLaunchKernelGGL((k_gather_grad<P, false, float>), dim3(blocks), dim3(256), 0, s,
                         (const float*)pos, n_total, offsets, (const float*)b.grid, g, w, (float*)grad);
  } else {
    if (g.il)
      hipLaunchKernelGGL((k_gather_grad<P, true, double>), dim3(blocks), dim3(256), 0, s,
                         (const double*)pos, n_total, offsets, (const float*)b.grid, g, w,
                         (double*)grad);
    else
      hipLaunchKernelGGL((k_gather_grad<P, false, double>), dim3(blocks), dim3(256), 0, s,
                         (const double*)pos, n_total, offsets, (const float*)b.grid, g, w,
                         (double*)grad);
  }
}

hipError_t launch_gather_grad(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                              int64_t n_total, const float* w, const Buffers& b, void* grad,
                              hipStream_t s) {
  switch (g.order) {
    case 1: dispatch_gather<1>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
    case 2: dispatch_gather<2>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
    case 3: dispatch_gather<3>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
    case 4: dispatch_gather<4>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
    case 5: dispatch_gather<5>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
    default: dispatch_gather<6>(g, pos, dt, offsets, n_total, w, b, grad, s); break;
  }
  return hipGetLastError();
}

}  // namespace fsest
