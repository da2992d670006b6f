// Bucket sort of the particles by 4^3-cell bucket of their first stencil
// cell (the deposit's input order), the per-set counts and mass sums, and small fill/scan utilities.
//
// Design (gfx950): by default two levels without device-scope atomics
// (per-workgroup LDS histograms over super-buckets, a scan, a super-bucket
// scatter, then one workgroup per super-bucket sorting its buckets in LDS);
// a single-level counting sort with device-scope atomics is the fallback.
// The positions are read only here: the sorted output is one 16-byte record
// per particle (particles.hpp: floor cells, interlacing steps and 24-bit
// offsets), so the deposit does all its work in integers and float32.
#include "particles.hpp"

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
// Per set, weight_slices(batch) workgroups each sum w and w^2 over a fixed
// slice of the set's particles (strided per thread, then a fixed tree over
// the workgroup), and a second pass adds the slices in order: the totals
// depend on the batch size only, not on scheduling.  The largest mass goes to stats[4] (non-negative
// floats order like their bit patterns) and any negative, NaN or infinite
// mass sets stats[5].
constexpr int kWThreads = 256;

__global__ __launch_bounds__(kWThreads) void k_weight_stats(const float* __restrict__ w,
                                                            const int64_t* __restrict__ offsets,
                                                            int64_t n_total,
                                                            double* __restrict__ wpart,
                                                            uint32_t* __restrict__ stats) {
  __shared__ double sa[kWThreads / 64], sb[kWThreads / 64];
  const int m = blockIdx.y, slice = blockIdx.x, ns = gridDim.x;
  const int64_t j0 = offsets ? offsets[m] : 0, j1 = offsets ? offsets[m + 1] : n_total;
  const int64_t len = j1 - j0;
  const int64_t s0 = j0 + len * slice / ns, s1 = j0 + len * (slice + 1) / ns;
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
    double* dst = wpart + 2 * ((int64_t)m * ns + slice);
    dst[0] = ta;
    dst[1] = tb;
  }
}

__global__ void k_weight_final(const double* __restrict__ wpart, int batch, int ns,
                               double* __restrict__ norm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= batch) return;
  double ta = 0.0, tb = 0.0;
  for (int i = 0; i < ns; ++i) {
    ta += wpart[2 * ((int64_t)m * ns + i)];
    tb += wpart[2 * ((int64_t)m * ns + i) + 1];
  }
  norm[2 * m] = ta;
  norm[2 * m + 1] = tb;
}

hipError_t launch_weight_stats(const float* w, const int64_t* offsets, int64_t n_total, int batch,
                               double* wpart, double* norm, uint32_t* stats, hipStream_t s) {
  hipError_t e = launch_fill_u32(stats + 4, 2, 0u, s);
  if (e != hipSuccess) return e;
  const int ns = weight_slices(batch);
  hipLaunchKernelGGL(k_weight_stats, dim3(ns, batch), dim3(kWThreads), 0, s, w, offsets,
                     n_total, wpart, stats);
  hipLaunchKernelGGL(k_weight_final, dim3((batch + 63) / 64), dim3(64), 0, s, wpart, batch, ns,
                     norm);
  return hipGetLastError();
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
    const int bx = bucket_of(grid_coord(x, g.box, g.inv), g);
    const int by = bucket_of(grid_coord(y, g.box, g.inv), g);
    const int bz = bucket_of(grid_coord(z, g.box, g.inv), g);
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

// The two-level sort carries a particle's bucket inside its super-bucket
// (12 bits) between its two passes in the free upper bytes of the record's
// z and w words.
__device__ __forceinline__ uint4 with_fine(uint4 r, uint32_t fine) {
  r.z |= (fine & 255u) << 24;
  r.w |= (fine >> 8) << 24;
  return r;
}
__device__ __forceinline__ uint32_t fine_of(uint4 r) { return (r.z >> 24) | ((r.w >> 24) << 8); }
__device__ __forceinline__ uint4 without_fine(uint4 r) {
  r.z &= kFracMask;
  r.w &= kFracMask;
  return r;
}

template <typename TP>
__global__ __launch_bounds__(256) void k_bucket_scatter(const TP* __restrict__ pos, int64_t n_total,
                                                        const int64_t* __restrict__ offsets, Geom g,
                                                        const uint32_t* __restrict__ boff,
                                                        const uint32_t* __restrict__ rank,
                                                        uint4* __restrict__ recs,
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
  const int bx = bucket_of(ux, g);
  const int by = bucket_of(uy, g);
  const int bz = bucket_of(uz, g);
  const uint32_t key = (uint32_t)(((int64_t)mock * g.nb + bx) * g.nb + by) * g.nb + bz;
  const int64_t dst = (int64_t)boff[key] + rank[j];
  recs[dst] = particle_record(ux, uy, uz, g);
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
                       n_total, offsets, g, b.boff, b.rank, b.recs, w, b.sw, b.stats);
  else
    hipLaunchKernelGGL(k_bucket_scatter<double>, dim3(pblocks), dim3(256), 0, s,
                       (const double*)pos, n_total, offsets, g, b.boff, b.rank, b.recs, w, b.sw,
                       b.stats);
  return hipGetLastError();
}

// ---- two-level sort without device-scope atomics
// Super-buckets are cubes of g.fb^3 buckets (g.nsup of them).  (A) each of
// nblk workgroups histograms a contiguous chunk of particles over the
// super-buckets in LDS; (B) the histograms, laid out super-major, are
// scanned, giving every (super-bucket, workgroup) pair its output offset;
// (C) each workgroup re-reads its chunk and moves every particle's record
// into its super-bucket segment, ranking with LDS counters, and writes the
// particle's bucket inside the super-bucket beside it (2 bytes); (D) one
// workgroup per super-bucket counts its particles per bucket from those
// 2-byte indices, writes the bucket offsets and counts, and moves the
// records into bucket order.  Buckets are therefore contiguous in z inside a super-bucket;
// the deposit splits its bucket runs at super-bucket boundaries.
constexpr int kSortThreads = 1024;
constexpr int kSortBatch = 4;  // particles per thread whose loads are in flight together
constexpr int kFineBlocks = 512;  // workgroups of the bucket pass (two per CU of an MI355X)

__device__ __forceinline__ void particle_buckets(double ux, double uy, double uz, const Geom& g,
                                                 int& bx, int& by, int& bz) {
  bx = bucket_of(ux, g);
  by = bucket_of(uy, g);
  bz = bucket_of(uz, g);
}

// x / fb for a bucket index x (< 2^16): floor(x m / 2^32) with m = floor(2^32 / fb) + 1
// is exact there, since the error x (m fb - 2^32) / (fb 2^32) < 2^-16 < 1/fb
__device__ __forceinline__ int div_fb(int x, const Geom& g) {
  return g.fb == 1 ? x : (int)__umulhi((uint32_t)x, g.fb_mul);
}

__device__ __forceinline__ int super_of(int mock, int bx, int by, int bz, const Geom& g) {
  return ((mock * g.sa + div_fb(bx, g)) * g.sa + div_fb(by, g)) * g.sa + div_fb(bz, g);
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
  // the sets this chunk spans
  const int mlo = j0 < j1 ? mock_of(offsets, g.batch, j0) : 0;
  const int mhi = j0 < j1 ? mock_of(offsets, g.batch, j1 - 1) : 0;
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
        atomicAdd(&hist[super_of(mlo == mhi ? mlo : mock_in(offsets, mlo, mhi, j), bx, by, bz, g)], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < g.nsup; i += kSortThreads)
    hsup[(int64_t)blockIdx.x * g.nsup + i] = hist[i];
}

template <typename TP>
__global__ __launch_bounds__(kSortThreads) void k_sort_super(
    const TP* __restrict__ pos, int64_t n_total, const int64_t* __restrict__ offsets, Geom g,
    int64_t chunk, const uint32_t* __restrict__ hoff, const uint32_t* __restrict__ base,
    uint4* __restrict__ trec,
    uint16_t* __restrict__ tfine, const float* __restrict__ w, float* __restrict__ tw) {
  __shared__ uint32_t cur[kMaxSuper];
  for (int i = threadIdx.x; i < g.nsup; i += kSortThreads)
    cur[i] = base[i] + hoff[(int64_t)blockIdx.x * g.nsup + i];
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = (j0 + chunk < n_total) ? j0 + chunk : n_total;
  const int mlo = j0 < j1 ? mock_of(offsets, g.batch, j0) : 0;
  const int mhi = j0 < j1 ? mock_of(offsets, g.batch, j1 - 1) : 0;
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
        const int sup = super_of(mlo == mhi ? mlo : mock_in(offsets, mlo, mhi, j), bx, by, bz, g);
        const int fx = bx - div_fb(bx, g) * g.fb, fy = by - div_fb(by, g) * g.fb;
        const int fz = bz - div_fb(bz, g) * g.fb;
        const uint32_t fine = (uint32_t)((fx * g.fb + fy) * g.fb + fz);
        const uint32_t p = atomicAdd(&cur[sup], 1u);
        trec[p] = with_fine(particle_record(ux, uy, uz, g), fine);
        tfine[p] = (uint16_t)fine;
        if (w) tw[p] = w[j];
      }
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_fine(
    const uint4* __restrict__ trec, const uint16_t* __restrict__ tfine, Geom g,
    const uint32_t* __restrict__ base, uint4* __restrict__ recs, uint32_t* __restrict__ boff,
    uint32_t* __restrict__ bcnt, uint32_t* __restrict__ stats, const float* __restrict__ tw,
    float* __restrict__ sw) {
  constexpr int kPer = kFineMax * kFineMax * kFineMax / kSortThreads;  // buckets per thread
  __shared__ uint32_t hist[kFineMax * kFineMax * kFineMax];
  __shared__ uint32_t wtot[kSortThreads / 64];
  __shared__ int next_sup;
  // a fixed grid takes the super-buckets in order from a counter (stats[3],
  // zeroed with the sort's statistics), so that the ones in flight are
  // neighbours and uneven ones balance
  for (;;) {
  if (threadIdx.x == 0) next_sup = (int)atomicAdd(&stats[3], 1u);
  __syncthreads();  // also: the previous super-bucket's scatter is done
  const int sup = next_sup;
  if (sup >= g.nsup) break;
  const int nf = g.fb * g.fb * g.fb;
  const uint32_t seg0 = base[sup], seg1 = base[sup + 1];
  for (int i = threadIdx.x; i < nf; i += kSortThreads) hist[i] = 0u;
  __syncthreads();
  // the histogram reads the 2-byte bucket indices, not the records
  for (uint32_t ib = seg0 + threadIdx.x; ib < seg1; ib += kSortBatch * kSortThreads) {
    uint32_t f[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const uint32_t i = ib + q * kSortThreads;
      f[q] = (i < seg1) ? (uint32_t)tfine[i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q)
      if (ib + q * kSortThreads < seg1) atomicAdd(&hist[f[q]], 1u);
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
    uint4 r[kSortBatch];
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      const uint32_t i = ib + q * kSortThreads;
      if (i < seg1) r[q] = trec[i];
    }
#pragma unroll
    for (int q = 0; q < kSortBatch; ++q) {
      if (ib + q * kSortThreads < seg1) {
        const uint32_t p = seg0 + atomicAdd(&hist[fine_of(r[q])], 1u);
        recs[p] = without_fine(r[q]);
        if (tw) sw[p] = scaled_mass(tw, ib + q * kSortThreads, stats);
      }
    }
  }
  }
}

// The histograms are stored block-major (h[b][s], b < nblk, s < nsup, so
// that every pass reads and writes them in whole rows).  Per super-bucket s
// this replaces h[b][s] by its exclusive prefix over the blocks and writes
// the column total to tot[s].  A workgroup takes 64 consecutive s (one per
// lane) and splits the blocks over its 16 waves.
constexpr int kColThreads = 1024;
constexpr int kColWaves = kColThreads / 64;

__global__ __launch_bounds__(kColThreads) void k_sup_colscan(uint32_t* __restrict__ h, int nsup,
                                                             int nblk, uint32_t* __restrict__ tot) {
  __shared__ uint32_t part[kColWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sup = blockIdx.x * 64 + lane;
  const int b0 = nblk * wave / kColWaves, b1 = nblk * (wave + 1) / kColWaves;
  uint32_t sum = 0;
  if (sup < nsup)
    for (int b = b0; b < b1; ++b) sum += h[(int64_t)b * nsup + sup];
  part[wave][lane] = sum;
  __syncthreads();
  uint32_t run = 0, all = 0;
  for (int w = 0; w < kColWaves; ++w) {
    const uint32_t v = part[w][lane];
    run += (w < wave) ? v : 0u;
    all += v;
  }
  if (sup < nsup) {
    for (int b = b0; b < b1; ++b) {
      const uint32_t v = h[(int64_t)b * nsup + sup];
      h[(int64_t)b * nsup + sup] = run;
      run += v;
    }
    if (wave == 0) tot[sup] = all;
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
  // per-block offsets inside each super-bucket, then the super-bucket starts
  // (base[nsup] = n_total) after the kMaxSortBlocks rows of histograms
  uint32_t* base = b.hsup + (size_t)g.nsup * kMaxSortBlocks;
  hipLaunchKernelGGL(k_sup_colscan, dim3((g.nsup + 63) / 64), dim3(kColThreads), 0, s, b.hsup,
                     g.nsup, nblk, base);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the scan's largest-entry output is not a bucket count here
  if ((e = scan_in_place(base, (size_t)g.nsup + 1, b.scan_tmp, b.stats + 2, s)) != hipSuccess)
    return e;
  // the per-particle ranks of the atomic sort are not used here: their
  // buffer holds each particle's bucket inside its super-bucket (2 bytes)
  uint16_t* tfine = reinterpret_cast<uint16_t*>(b.rank);
  hipLaunchKernelGGL(k_sort_super<TP>, dim3(nblk), dim3(kSortThreads), 0, s, pos, n_total,
                     offsets, g, chunk, b.hsup, (const uint32_t*)base, b.trecs, tfine, w, b.tw);
  hipLaunchKernelGGL(k_sort_fine, dim3(g.nsup < kFineBlocks ? g.nsup : kFineBlocks), dim3(kSortThreads), 0, s, (const uint4*)b.trecs,
                     (const uint16_t*)tfine, g, (const uint32_t*)base, b.recs,
                     b.boff, b.bcnt, b.stats, w ? b.tw : nullptr, b.sw);
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

}  // namespace fsest
