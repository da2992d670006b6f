// Direct summation of the Fourier-space density (Sec. 2.2, eq. deltaDS):
//   delta_DS(m) = N_P^-1 sum_j exp(-2 pi i m . x_j / L)
// at every half-space mode of the grid (m_x, m_y in [-N/2, N/2], m_z in
// [0, N/2]), the alias-free reference the FFT estimator is compared with.
// With masses w_j the sum is W^-1 sum_j w_j exp(...), W = sum_j w_j.
//
// Design (gfx950, ALU-bound, O(N_P N^3 / 2)):
//  * each particle's position becomes three 32-bit fixed-point phases
//    q_a = floor(wrap(x_a) / L * 2^32), so m . x / L mod 1 is the exact
//    integer m_x q_x + m_y q_y + m_z q_z mod 2^32 (phase error < 2^-32 m);
//  * a thread owns one (m_x, m_y) and MZ consecutive m_z: per particle one
//    accurate sincos of the first phase, then complex steps by
//    exp(-2 pi i q_z / 2^32) for the others; particles are staged in LDS in
//    chunks and summed in FP32 per chunk, then in FP64.  MZ (8, 11, 13 or
//    16) is the one that leaves fewest idle slots in a row's N/2 + 1 modes
//    (11 for N = 64, 13 for N = 128), so the sincos is shared by more terms;
//  * particles are split into S slices (a grid dimension) for parallelism;
//    a fixed-order FP64 reduction over the slices gives deterministic output.
#include <mutex>

#include "fsest_internal.hpp"

namespace fsest {

constexpr int kDirThreads = 256;
constexpr int kDirChunk = 256;   // particles per LDS chunk

template <typename TP>
__global__ void k_dir_prep(const TP* __restrict__ pos, int64_t n, double box,
                           uint32_t* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int a = 0; a < 3; ++a) {
    const double t = wrap_coord((double)pos[3 * j + a], box) / box;  // [0, 1]
    const double s = t * 4294967296.0;
    q[3 * j + a] = (s >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)s;
  }
}

// partial[slice][mode] (complex128) of the half spectrum, mode index
// (ix * N + iy) * (N/2 + 1) + mz with ix, iy the FFT indices
template <bool WT, int MZ>
__global__ __launch_bounds__(kDirThreads) void k_direct(const uint32_t* __restrict__ q, int64_t n,
                                                        int ngrid, int nslices,
                                                        const float* __restrict__ w,
                                                        double* __restrict__ partial) {
  __shared__ uint32_t sq[3 * kDirChunk];
  __shared__ float2 sstep[kDirChunk];
  __shared__ float swt[WT ? kDirChunk : 1];
  const int nh = ngrid / 2 + 1;
  const int nzb = (nh + MZ - 1) / MZ;
  const int64_t nthreads_modes = (int64_t)ngrid * ngrid * nzb;
  const int64_t tid = (int64_t)blockIdx.x * kDirThreads + threadIdx.x;
  const bool active = tid < nthreads_modes;
  const int zb = (int)(tid % nzb);
  const int iy = (int)((tid / nzb) % ngrid);
  const int ix = (int)(tid / ((int64_t)nzb * ngrid));
  const int mx = (ix <= ngrid / 2) ? ix : ix - ngrid;
  const int my = (iy <= ngrid / 2) ? iy : iy - ngrid;
  const int mz0 = zb * MZ;
  const int slice = blockIdx.y;
  const int64_t j0 = n * slice / nslices, j1 = n * (slice + 1) / nslices;

  double accr[MZ], acci[MZ];
#pragma unroll
  for (int r = 0; r < MZ; ++r) accr[r] = acci[r] = 0.0;

  for (int64_t c0 = j0; c0 < j1; c0 += kDirChunk) {
    const int cn = (int)((j1 - c0) < kDirChunk ? (j1 - c0) : kDirChunk);
    __syncthreads();  // previous chunk consumed
    for (int i = threadIdx.x; i < cn; i += kDirThreads) {
      const uint32_t qx = q[3 * (c0 + i) + 0], qy = q[3 * (c0 + i) + 1], qz = q[3 * (c0 + i) + 2];
      sq[3 * i + 0] = qx;
      sq[3 * i + 1] = qy;
      sq[3 * i + 2] = qz;
      float s, c;
      // exp(-2 pi i q_z / 2^32): sincospi of 2 q_z / 2^32 = q_z / 2^31
      sincospif((float)qz * 4.656612873077393e-10f, &s, &c);
      sstep[i] = make_float2(c, -s);
      if constexpr (WT) {
        const float v = w[c0 + i];
        swt[i] = (v >= 0.0f && v <= 3.402823466e38f) ? v : 0.0f;
      }
    }
    __syncthreads();
    if (active) {
      float fr[MZ], fi[MZ];
#pragma unroll
      for (int r = 0; r < MZ; ++r) fr[r] = fi[r] = 0.0f;
      for (int i = 0; i < cn; ++i) {
        const uint32_t qx = sq[3 * i + 0], qy = sq[3 * i + 1], qz = sq[3 * i + 2];
        const uint32_t ph = (uint32_t)mx * qx + (uint32_t)my * qy + (uint32_t)mz0 * qz;
        float s, c;
        sincospif((float)ph * 4.656612873077393e-10f, &s, &c);
        float er = c, ei = -s;
        if constexpr (WT) {
          er *= swt[i];
          ei *= swt[i];
        }
        const float2 st = sstep[i];
#pragma unroll
        for (int r = 0; r < MZ; ++r) {
          fr[r] += er;
          fi[r] += ei;
          const float tr = er * st.x - ei * st.y;
          ei = er * st.y + ei * st.x;
          er = tr;
        }
      }
#pragma unroll
      for (int r = 0; r < MZ; ++r) {
        accr[r] += fr[r];
        acci[r] += fi[r];
      }
    }
  }
  if (!active) return;
  const int64_t nmodes = (int64_t)ngrid * ngrid * nh;
  double* out = partial + 2 * nmodes * slice;
  const int64_t base = ((int64_t)ix * ngrid + iy) * nh;
#pragma unroll
  for (int r = 0; r < MZ; ++r) {
    const int mz = mz0 + r;
    if (mz < nh) {
      out[2 * (base + mz)] = accr[r];
      out[2 * (base + mz) + 1] = acci[r];
    }
  }
}

// norm (with masses): (W, sum w^2) from the mass-sum pass, stats[5] set for an
// invalid mass (then every mode is NaN)
__global__ void k_dir_reduce(const double* __restrict__ partial, int64_t nmodes, int nslices,
                             double inv_n, const double* __restrict__ norm,
                             const uint32_t* __restrict__ stats, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nmodes) return;
  double s = 0.0;
  for (int k = 0; k < nslices; ++k) s += partial[2 * nmodes * k + i];
  if (norm) out[i] = stats[5] ? __builtin_nan("") : s / norm[0];
  else out[i] = s * inv_n;
}

// m_z per thread: of 8, 11, 13 and 16 the one with the fewest idle slots in
// a row's N/2 + 1 modes, the larger on a tie
static int direct_mz(int ngrid) {
  const int nh = ngrid / 2 + 1;
  const int cand[4] = {8, 11, 13, 16};
  int best = 8, idle = 1 << 30;
  for (int c : cand) {
    const int w = (nh + c - 1) / c * c - nh;
    if (w < idle || (w == idle && c > best)) {
      best = c;
      idle = w;
    }
  }
  return best;
}

int direct_slices(int ngrid, int64_t n) {
  const int nh = ngrid / 2 + 1;
  const int mz = direct_mz(ngrid);
  const int64_t threads = (int64_t)ngrid * ngrid * ((nh + mz - 1) / mz);
  int64_t s = (2 * 256 * 1024 + threads - 1) / threads;
  const int64_t by_n = (n + kDirChunk - 1) / kDirChunk;
  if (s > by_n) s = by_n;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

// workspace: fixed-point phases, the mass sums (partials, totals, flags),
// then the per-slice partial spectra
constexpr size_t kDirMassBytes = 256 * ((2 * kWSlicesMax * 8 + 2 * 8 + 64 * 4 + 255) / 256);

// Static workspace of the allocation-free entry point.  In host code the
// name `scratch` only stands for the symbol: its device address comes from
// hipGetSymbolAddress, looked up once per device with that device current
// and kept in g_scratch_ptr; only that pointer is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kDirectStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t direct_static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* direct_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

size_t direct_workspace(int ngrid, int64_t n) {
  const int64_t nmodes = (int64_t)ngrid * ngrid * (ngrid / 2 + 1);
  const size_t qbytes = ((size_t)n * 3 * sizeof(uint32_t) + 255) / 256 * 256;
  return qbytes + kDirMassBytes + (size_t)direct_slices(ngrid, n) * nmodes * 2 * sizeof(double);
}

hipError_t launch_direct(const Geom& g, const void* pos, est_dtype dt, int64_t n, const float* w,
                         void* ws, double* out, hipStream_t s) {
  const int ngrid = g.n;
  const int nh = ngrid / 2 + 1;
  const int64_t nmodes = (int64_t)ngrid * ngrid * nh;
  const int nslices = direct_slices(ngrid, n);
  uint32_t* q = (uint32_t*)ws;
  char* mass = (char*)ws + ((size_t)n * 3 * sizeof(uint32_t) + 255) / 256 * 256;
  double* wpart = (double*)mass;
  double* norm = wpart + 2 * kWSlicesMax;
  uint32_t* stats = (uint32_t*)(norm + 2);
  double* partial = (double*)(mass + kDirMassBytes);
  if (w) {
    hipError_t e = launch_weight_stats(w, nullptr, n, 1, wpart, norm, stats, s);
    if (e != hipSuccess) return e;
  }
  const unsigned pb = (unsigned)((n + 255) / 256);
  if (dt == EST_F32)
    hipLaunchKernelGGL(k_dir_prep<float>, dim3(pb), dim3(256), 0, s, (const float*)pos, n, g.box, q);
  else
    hipLaunchKernelGGL(k_dir_prep<double>, dim3(pb), dim3(256), 0, s, (const double*)pos, n, g.box,
                       q);
  const int mz = direct_mz(ngrid);
  const int64_t threads = (int64_t)ngrid * ngrid * ((nh + mz - 1) / mz);
  const dim3 grid((unsigned)((threads + kDirThreads - 1) / kDirThreads), nslices);
#define FSEST_DIRECT_CASE(MZV)                                                                  \
  case MZV:                                                                                     \
    if (w)                                                                                      \
      hipLaunchKernelGGL((k_direct<true, MZV>), grid, dim3(kDirThreads), 0, s, q, n, ngrid,     \
                         nslices, w, partial);                                                  \
    else                                                                                        \
      hipLaunchKernelGGL((k_direct<false, MZV>), grid, dim3(kDirThreads), 0, s, q, n, ngrid,    \
                         nslices, w, partial);                                                  \
    break;
  switch (mz) {
    FSEST_DIRECT_CASE(8)
    FSEST_DIRECT_CASE(11)
    FSEST_DIRECT_CASE(13)
    default: FSEST_DIRECT_CASE(16)
  }
#undef FSEST_DIRECT_CASE
  hipLaunchKernelGGL(k_dir_reduce, dim3((unsigned)((2 * nmodes + 255) / 256)), dim3(256), 0, s,
                     partial, nmodes, nslices, 1.0 / (double)n, w ? norm : nullptr, stats, out);
  return hipGetLastError();
}

}  // namespace fsest
