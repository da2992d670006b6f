// Internal declarations shared by the HIP translation units of libfsest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "../../include/fsest.h"

namespace fsest {

constexpr int kBucket = 4;      // bucket edge in cells (particles sorted by bucket)
constexpr int kTileMax = 16;    // deposit tile edge in cells (LDS-resident)
constexpr int kMaxBins = 512;   // largest n_bins (N / 2 at N = 1024)
constexpr int kMaxBinBlocks = 2048;  // upper bound of P(k) reduction blocks per set
constexpr int kFineMax = 16;    // buckets per super-bucket edge (two-level sort)
constexpr int kMaxSuper = 8192; // super-buckets one workgroup histograms in LDS
constexpr int kMaxSortBlocks = 1024;  // workgroups of the super-bucket passes
constexpr int kWSlicesMax = 1024;  // workgroups per set of the mass-sum pass, at most
// workgroups per set of the mass-sum pass: ~2048 in all, 16 .. 1024 per set
__host__ __device__ inline int weight_slices(int batch) {
  const int s = 2048 / batch;
  return s < 16 ? 16 : (s > kWSlicesMax ? kWSlicesMax : s);
}

// Geometry and per-call constants that device code needs.
struct Geom {
  int n;          // N
  int nz;         // complex length of the contiguous axis: N (interlaced) or N/2
  int order;      // p
  int il;         // grids packed in pairs as complex (interlacing code >= 1)
  int code;       // interlacing code: 0 one grid, 1 the pair {0, (1,1,1)/2}, 2 the four
                  // face-centred half-cell shifts, 3 all eight half-cell shifts
  int ng;         // grids per set: 1, 2, 4, 8
  int npair;      // complex grids (slabs) per set: max(1, ng / 2); slab = set * npair + q
  int batch;
  int nb;         // buckets per axis = N / kBucket
  int tile;       // deposit tile edge
  int fb;         // buckets per super-bucket edge: min(kFineMax, nb)
  uint32_t fb_mul;  // floor(2^32 / fb) + 1 (fb >= 2): x / fb = umulhi(x, fb_mul) for x < 2^16
  int sa;         // super-buckets per axis: nb / fb
  int nsup;       // batch * sa^3 (two-level sort when <= kMaxSuper)
  double box;     // L
  double inv;     // fl64(N / L)
  int64_t ps;     // complex elements between consecutive x planes: N*nz plus
                  // a pad that breaks the power-of-two stride of the x pass
};

// Shift mask of grid j (bit a: sampled at u_a + 1/2); grids 2q and 2q+1 share
// slab q as real and imaginary parts.
__host__ __device__ inline int grid_mask(int code, int j) {
  if (code == 1) return j ? 7 : 0;
  if (code == 2) return j == 0 ? 0 : (j == 1 ? 3 : (j == 2 ? 5 : 6));
  return code == 3 ? j : 0;
}

// float index of real-grid cell (x, y, z) of set `mock` (plane stride ps
// complex = 2 ps floats; without interlacing the N^3 reals are packed two per
// complex element along z, so a row of N floats is nz = N/2 complex)
__device__ __forceinline__ int64_t real_cell_index(const Geom& g, int mock, int x, int y, int z) {
  return 2 * (((int64_t)mock * g.n + x) * g.ps) + (int64_t)y * g.n + z;
}
// complex element (x, y, z) of set `mock`, z < nz
__device__ __forceinline__ int64_t complex_index(const Geom& g, int mock, int x, int y, int z) {
  return ((int64_t)mock * g.n + x) * g.ps + (int64_t)y * g.nz + z;
}

// Work buffers carved out of the caller's workspace.
struct Buffers {
  float2* grid;            // batch * N * N * nz complex (rho1 + i rho2, or packed reals)
  uint4* recs;             // max_particles 16-byte particle records, bucket order
  uint32_t* rank;          // max_particles
  uint32_t* boff;          // batch * nb^3 + 1 bucket start offsets (key order)
  uint32_t* bcnt;          // batch * nb^3 bucket counts
  uint4* trecs;            // max_particles records in super-bucket order (two-level sort)
  uint32_t* hsup;          // kMaxSortBlocks x nsup block-major histograms / offsets,
                           // then the nsup + 1 super-bucket starts
  uint32_t* scan_tmp;      // scan block sums
  uint32_t* stats;         // [0] largest bucket count of the last sort, [1] tile counter,
                           // [4] largest mass (float bits), [5] nonzero if a mass is
                           // negative or not finite, [6] fraction bits of the
                           // deposit's 32-bit fixed point
  float2* tw_n;            // exp(-2 pi i n / N)
  float2* tw_nz;           // exp(-2 pi i n / nz)
  float* inv_w2;           // 1 / W_1D(m(i))^2 for FFT index i (N entries)
  float* win1;             // W_1D(m(i)) for FFT index i (N entries)
  float2* phase;           // exp(+i pi s / N), s = 0..2N-1
  double* partials;        // batch * kMaxBinBlocks * kMaxBins
  int64_t* mode_n;         // kMaxBins
  double* mode_k;          // kMaxBins
  int64_t* np;             // batch particle counts
  double* norm;            // batch x (W, sum w^2): total mass and sum of squared masses
                           // (N_P, N_P for equal masses)
  float* sw;               // max_particles masses / largest mass, bucket order (weighted handles)
  float* tw;               // max_particles masses in super-bucket order (weighted, two-level)
  double* wpart;           // batch x weight_slices(batch) x 2 partial mass sums (weighted)
  float2* cbuf;            // batch x N x N x (N/2+1) combined C(m) (interlace codes 2, 3)
  double* coef;            // batch * kMaxBins adjoint coefficients
  uint64_t* mode_partials_n;  // kMaxBinBlocks * kMaxBins
  double* mode_partials_k;    // kMaxBinBlocks * kMaxBins
};

// Launch shapes chosen per handle (the autotuner changes them).
struct Tune {
  int cols_c = 16;        // lines per workgroup of the strided FFT passes
  int bin_blocks = 1024;  // reduction workgroups per set in the fused P(k) pass
  int dep_threads = 0;    // threads per deposit workgroup (0: chosen per kernel)
  int dep_narrow = 1;     // 32-bit fixed point when provably safe (else 64-bit)
  int dep_xcd = 1;        // consecutive deposit tiles on one XCD (shared L2)
  int cus = 256;          // compute units of the handle's device (set at create)
};

// Device helper: wrap one float64 coordinate into [0, L) with the fixed
// operation sequence x - L floor(x/L), +L if negative, -L if >= L, and 0 for
// anything left outside [0, L) (also NaN).
__device__ __forceinline__ double wrap_coord(double x, double box) {
#pragma clang fp contract(off)
  if (x >= 0.0 && x < box) return x;  // x - L*floor(x/L) == x exactly here
  double q = floor(x / box);
  double xw = x - q * box;
  if (xw < 0.0) xw = xw + box;
  if (xw >= box) xw = xw - box;
  if (!(xw >= 0.0 && xw < box)) xw = 0.0;
  return xw;
}

__device__ __forceinline__ double grid_coord(double x, double box, double inv) {
#pragma clang fp contract(off)
  return wrap_coord(x, box) * inv;
}

// ---- launchers (return hipError_t of the last launch) ----
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
// particle counts per set; norm = (N_P, N_P) per set (equal masses)
hipError_t launch_set_counts(const int64_t* offsets, int64_t n_total, int batch, int64_t* np,
                             double* norm, hipStream_t s);
// masses w (original order): norm = (W, sum w^2) per set in a fixed summation
// order, stats[4] = largest mass, stats[5] = flag for invalid masses
hipError_t launch_weight_stats(const float* w, const int64_t* offsets, int64_t n_total, int batch,
                               double* wpart, double* norm, uint32_t* stats, hipStream_t s);
// w: masses in original order (null: equal masses); their bucket-order
// copy, divided by the largest mass, goes to b.sw
hipError_t launch_sort(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                       int64_t n_total, const float* w, const Buffers& b, hipStream_t s);
// from the sort's records (any position type); weighted: read b.sw and
// scale the grids by the largest mass
hipError_t launch_deposit(const Geom& g, const Buffers& b, const Tune& tu, bool weighted,
                          hipStream_t s);
hipError_t launch_copy_grid(const Geom& g, const Buffers& b, int which, int mock, float* dst,
                            hipStream_t s);
hipError_t launch_gather_grad(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                              int64_t n_total, const float* w, const Buffers& b, void* grad,
                              hipStream_t s);

hipError_t launch_tables(const Geom& g, const Buffers& b, hipStream_t s);
// direction: -1 forward, +1 inverse.  axis 0 = x (stride N*nz), 1 = y (stride nz), 2 = z (rows).
hipError_t launch_fft_axis(const Geom& g, float2* data, int axis, int dir, int batch,
                           int nz_len, const float2* tw_axis, const Tune& tu, hipStream_t s);
// one axis of transforms of length L (any 2^a 3^b 5^c up to 1024) on a
// buffer: contiguous rows (row r at (r / rows_per_plane) plane_stride +
// (r % rows_per_plane) L), or strided lines (inner adjacent lines per outer
// block, c of them per workgroup); tw[n] = exp(-2 pi i n / L)
hipError_t launch_fft_rows_len(int L, float2* data, int64_t nrows, int rows_per_plane,
                               int64_t plane_stride, int dir, const float2* tw, hipStream_t s);
hipError_t launch_fft_cols_len(int L, float2* data, int64_t elem_stride, int64_t inner, int64_t outer,
                               int64_t outer_stride, int dir, int c, const float2* tw, hipStream_t s);
hipError_t launch_mode_table(const Geom& g, const Buffers& b, int n_dk, int n_bins, hipStream_t s);
// fused last-axis forward FFT (if do_fft) + interlace + deconvolve + shell sums + finalize
hipError_t launch_power(const Geom& g, const Buffers& b, const Tune& tu, bool do_fft, int n_dk,
                        int n_bins, int subtract_shot, double* k, double* p, int64_t* nmodes,
                        hipStream_t s);
// adjoint: coefficients from dL/dP, then fused z-forward, gradient spectrum, z-inverse
hipError_t launch_adjoint_spectrum(const Geom& g, const Buffers& b, const Tune& tu,
                                   const double* dldp, int n_dk, int n_bins, hipStream_t s);
// adjoint for more than two grids: from the stored spectra (after the z pass)
// to the gradient spectra of every slab; the inverse z, y, x passes follow
hipError_t launch_multi_adjoint(const Geom& g, const Buffers& b, const double* dldp, int n_dk,
                                int n_bins, hipStream_t s);
hipError_t launch_sample_delta(const Geom& g, const Buffers& b, int mock, const int32_t* modes,
                               int64_t n, double* out, hipStream_t s);
hipError_t launch_export_delta(const Geom& g, const Buffers& b, int mock, double* out,
                               hipStream_t s);
// P = V sum_shell w Re(a conj(b)) / N_b - shot over half spectra a, b (b null: |a|^2)
hipError_t launch_spectrum_power(const Geom& g, const Buffers& b, const double* a, const double* bb,
                                 int n_dk, int n_bins, double shot, double* k, double* p,
                                 int64_t* nmodes, hipStream_t s);
// direct summation (eq. deltaDS) over every half-space mode
size_t direct_workspace(int ngrid, int64_t n);
// the allocation-free entry point's static workspace (64 MiB per device):
// looked up once per device (hipGetSymbolAddress with that device current),
// then its device address; null before a successful init on that device
constexpr size_t kDirectStaticBytes = (size_t)64 << 20;
hipError_t direct_static_scratch_init(int device);
void* direct_static_scratch(int device);
// w: masses (null: equal masses), normalised by their sum
hipError_t launch_direct(const Geom& g, const void* pos, est_dtype dt, int64_t n, const float* w,
                         void* ws,
                         double* out, hipStream_t s);
// ---- FFT-shell bispectrum (bispec.hip)
// One call's plan: band radius R (every mode of shells 1..n_bins has
// |m_a| <= R), the alias-free grid M > 3R, Q shell pairs, slabs of S
// x-planes, points per LDS chunk pc, tile jobs, job groups and point ranges
// of the triple-sum launch, and the byte offsets of the regions of the
// caller's bispectrum workspace.
struct BsPlan {
  int R, M, Q, S, nslab, pc, ngroups, nranges;
  int64_t npts, njobs;
  size_t off_tw, off_band, off_slab, off_jobs, off_tmap, off_part, off_run, bytes;
};
// jobs of every ordered triple b1 >= b2 >= b3 of shells 1..n_bins
int64_t bs_max_jobs(int n_bins);
// false if no grid of the form 2^a 3^b 5^c between 3R and min(N, 1024) exists
bool bs_plan(int n, int n_dk, int n_bins, int64_t njobs, int64_t n_tri, BsPlan* pl);
// the tile jobs (int32 x 4 each: d, r0, c0, 0) of a triangle list and each
// triangle's (job, entry) pair
void bs_jobs(const int32_t* tri, int64_t n_tri, std::vector<int32_t>& jobs,
             std::vector<int32_t>& tmap);
// twiddles of length M and the cube of delta(m), |m_a| <= R
hipError_t launch_bs_setup(const Geom& g, const Buffers& b, int mock, int n_dk, int n_bins,
                           const BsPlan& pl, char* bws, hipStream_t s);
// the fields of slab `slab_index` (delta, or the counts when `counts`)
hipError_t launch_bs_fields(int n_dk, int n_bins, const BsPlan& pl, char* bws, bool counts,
                            int slab_index, hipStream_t s);
// the slab's triple sums added to run (run cleared first for the first slab)
hipError_t launch_bs_triple(int n_bins, const BsPlan& pl, char* bws, bool first_slab, double* run,
                            hipStream_t s);
hipError_t launch_bs_finalize(const BsPlan& pl, char* bws, int64_t n_tri, double vol, double* bk,
                              double* ntri, hipStream_t s);

}  // namespace fsest
