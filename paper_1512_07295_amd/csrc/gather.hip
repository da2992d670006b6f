// Adjoint gather of the P(k) gradient (the transpose of the deposit, Sec. 2.3
// kernels differentiated): one thread per particle reads its stencils on
// every grid of its set.
#include "particles.hpp"

namespace fsest {

// ------------------------------------------------------------------ adjoint gather
// dL/dx_{j,alpha} = -(N/L) sum_a sum_{g in stencil_a} G_a(g) W'(s_alpha) prod_{beta != alpha} W(s_beta)
// where G_a = dL/drho_a sits in the grid buffer with the deposit's layout.
// IL: 0 one grid, 1 the interlaced pair, 2 the g.ng grids of interlace codes 2
// and 3 (grid gi: shift mask grid_mask(code, gi), component gi % 2 of slab
// gi / 2 of its set)
template <int P, int IL, typename TP>
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
  const int ngr = (IL == 2) ? g.ng : (IL ? 2 : 1);
#pragma unroll
  for (int gi = 0; gi < ngr; ++gi) {
    const int mk = (IL == 2) ? grid_mask(g.code, gi) : (gi ? 7 : 0);
    const int slab = (IL == 2) ? mock * g.npair + gi / 2 : mock;
    const int comp = gi & 1;
    int c[3][P];
    float wt[3][P], d[3][P];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double sh = ((mk >> ax) & 1) ? 0.5 : 0.0;
      stencil_1d<P>(u[ax] + sh, n, c[ax], wt[ax]);
      stencil_1d_deriv<P>(u[ax] + sh, d[ax]);
    }
    // float offsets of the stencil cells: x-plane (64-bit), then y and z
    // inside the plane (32-bit); a complex grid holds the grid as component
    // comp of each complex element, a packed real grid two reals per element
    int64_t xo[P];
    int yzo[P][P];
#pragma unroll
    for (int a = 0; a < P; ++a) xo[a] = 2 * (((int64_t)slab * n + c[0][a]) * g.ps);
#pragma unroll
    for (int bq = 0; bq < P; ++bq)
#pragma unroll
      for (int cq = 0; cq < P; ++cq)
        yzo[bq][cq] = IL ? 2 * (c[1][bq] * g.nz + c[2][cq]) + comp : c[1][bq] * n + c[2][cq];
#pragma unroll
    for (int a = 0; a < P; ++a) {
#pragma unroll
      for (int bq = 0; bq < P; ++bq) {
        // the x and y factors of the three derivative weights of this row
        const float fx = d[0][a] * wt[1][bq], fy = wt[0][a] * d[1][bq], fz = wt[0][a] * wt[1][bq];
#pragma unroll
        for (int cq = 0; cq < P; ++cq) {
          const float gv = grid[xo[a] + yzo[bq][cq]];
          const float t = gv * wt[2][cq];
          gx = __builtin_fmaf(fx, t, gx);
          gy = __builtin_fmaf(fy, t, gy);
          gz = __builtin_fmaf(fz * d[2][cq], gv, gz);
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

template <int P, int IL>
static void gather_t(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                     int64_t n_total, const float* w, const Buffers& b, void* grad, hipStream_t s) {
  const unsigned blocks = (unsigned)((n_total + 255) / 256);
  if (dt == EST_F32)
    hipLaunchKernelGGL((k_gather_grad<P, IL, float>), dim3(blocks), dim3(256), 0, s,
                       (const float*)pos, n_total, offsets, (const float*)b.grid, g, w, (float*)grad);
  else
    hipLaunchKernelGGL((k_gather_grad<P, IL, double>), dim3(blocks), dim3(256), 0, s,
                       (const double*)pos, n_total, offsets, (const float*)b.grid, g, w,
                       (double*)grad);
}

template <int P>
static void dispatch_gather(const Geom& g, const void* pos, est_dtype dt, const int64_t* offsets,
                            int64_t n_total, const float* w, const Buffers& b, void* grad,
                            hipStream_t s) {
  if (g.code >= 2) gather_t<P, 2>(g, pos, dt, offsets, n_total, w, b, grad, s);
  else if (g.code == 1) gather_t<P, 1>(g, pos, dt, offsets, n_total, w, b, grad, s);
  else gather_t<P, 0>(g, pos, dt, offsets, n_total, w, b, grad, s);
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
