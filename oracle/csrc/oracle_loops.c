/*
 * Plain FP64 loops of the oracle for large inputs (test infrastructure only;
 * see oracle/__init__.py).  They repeat, particle by particle, what
 * oracle/assign.py and oracle/direct.py compute with numpy:
 *
 *   stencil: even p -> first cell floor(u) - (p/2 - 1); odd p -> first cell
 *            floor(u + 1/2) - (p - 1)/2; p consecutive cells (mod N); weight
 *            W^(p)(cell - u) of Sec. 2.3 (CIC support |s| < 1; NGP weight 1;
 *            p = 5, 6: the centred B-spline's truncated-power sum).
 *   deposit: rho[g] += prod_axes W (eq. delgrid), grid index (x*N + y)*N + z.
 *   footprint DFT: F(m) = sum_j prod_axes sum_t w exp(-2 pi i m c / N).
 *
 * Inputs are grid coordinates u = wrap(x) * N / L computed by the numpy
 * oracle (plus 1/2 for the interlaced grid), so the cell choices are the
 * oracle's own.  The two sampling loops split the particles over OpenMP
 * threads; each thread sums its share and the shares are added in thread
 * order.  oracle_deposit_slabs splits the grid's x planes instead, which
 * keeps the serial loop's order of terms in every cell.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#define MAXP 6

/* 1/(p-1)! sum_k (-1)^k C(p,k) (s + p/2 - k)_+^(p-1) */
static double bspline(int p, double s) {
  double out = 0.0, c = 1.0, fact = 1.0;
  for (int i = 2; i < p; ++i) fact *= i;
  for (int k = 0; k <= p; ++k) {
    const double x = s + 0.5 * p - k;
    if (x > 0.0) out += ((k & 1) ? -c : c) * pow(x, p - 1);
    c = c * (p - k) / (k + 1);
  }
  return out / fact;
}

static double weight(int p, double s) {
  const double a = fabs(s);
  if (p > 4) return a < 0.5 * p ? bspline(p, s) : 0.0;
  switch (p) {
    case 1:
      return (s > -0.5 && s <= 0.5) ? 1.0 : 0.0;
    case 2:
      return a < 1.0 ? 1.0 - a : 0.0;
    case 3:
      if (a < 0.5) return 0.75 - s * s;
      if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
      return 0.0;
    default:
      if (a < 1.0) return (4.0 - 6.0 * s * s + 3.0 * a * a * a) / 6.0;
      if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
      return 0.0;
  }
}

static void stencil(double u, int p, int64_t n, int64_t* cell, double* w) {
  /* cell and w hold MAXP entries */
  const double first = (p % 2 == 0) ? floor(u) - (p / 2 - 1) : floor(u + 0.5) - (p - 1) / 2;
  for (int t = 0; t < p; ++t) {
    const double c = first + t;
    w[t] = (p == 1) ? 1.0 : weight(p, c - u);
    int64_t ci = ((int64_t)c) % n;
    if (ci < 0) ci += n;
    cell[t] = ci;
  }
}

/* rho (n^3, zeroed by the caller) += deposit of n_p particles at u (n_p x 3) */
void oracle_deposit(const double* u, int64_t n_p, int64_t n, int p, double* rho) {
  int64_t cx[MAXP], cy[MAXP], cz[MAXP];
  double wx[MAXP], wy[MAXP], wz[MAXP];
  for (int64_t j = 0; j < n_p; ++j) {
    stencil(u[3 * j + 0], p, n, cx, wx);
    stencil(u[3 * j + 1], p, n, cy, wy);
    stencil(u[3 * j + 2], p, n, cz, wz);
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b)
        for (int c = 0; c < p; ++c)
          rho[(cx[a] * n + cy[b]) * n + cz[c]] += wx[a] * wy[b] * wz[c];
  }
}

/* first cell of the p-point stencil of u (not reduced mod n), as in stencil() */
static int64_t first_cell(double u, int p) {
  const double first = (p % 2 == 0) ? floor(u) - (p / 2 - 1) : floor(u + 0.5) - (p - 1) / 2;
  return (int64_t)first;
}

/* The same sum as oracle_deposit with the x planes split among OpenMP
 * threads: thread t owns planes [n t / T, n (t+1) / T) and walks all
 * particles in order, adding only the stencil cells that lie in its planes.
 * Every cell therefore receives its terms in the serial loop's order with the
 * serial loop's arithmetic, so the grid equals oracle_deposit's bit for bit. */
void oracle_deposit_slabs(const double* u, int64_t n_p, int64_t n, int p, double* rho) {
#pragma omp parallel
  {
    const int64_t nt = omp_get_num_threads(), t = omp_get_thread_num();
    const int64_t x0 = n * t / nt, x1 = n * (t + 1) / nt;
    int64_t cx[MAXP], cy[MAXP], cz[MAXP];
    double wx[MAXP], wy[MAXP], wz[MAXP];
    for (int64_t j = 0; j < n_p; ++j) {
      /* cheap test first: does the x stencil meet this thread's planes? */
      const int64_t f = first_cell(u[3 * j + 0], p);
      int hit = 0;
      for (int a = 0; a < p; ++a) {
        int64_t c = (f + a) % n;
        if (c < 0) c += n;
        hit |= (c >= x0 && c < x1);
      }
      if (!hit) continue;
      stencil(u[3 * j + 0], p, n, cx, wx);
      stencil(u[3 * j + 1], p, n, cy, wy);
      stencil(u[3 * j + 2], p, n, cz, wz);
      for (int a = 0; a < p; ++a) {
        if (cx[a] < x0 || cx[a] >= x1) continue;
        for (int b = 0; b < p; ++b)
          for (int c = 0; c < p; ++c)
            rho[(cx[a] * n + cy[b]) * n + cz[c]] += wx[a] * wy[b] * wz[c];
      }
    }
  }
}

/* out_re/out_im[k] = sum_j prod_axes sum_t w exp(-2 pi i m_k c / N); the
 * phase of each integer cell is looked up in a per-mode, per-axis table */
void oracle_footprint_dft(const double* u, int64_t n_p, int64_t n, int p,
                          const int64_t* modes, int64_t n_modes,
                          double* out_re, double* out_im) {
  double* tr = (double*)malloc(sizeof(double) * (size_t)(n_modes * 3 * n));
  double* ti = (double*)malloc(sizeof(double) * (size_t)(n_modes * 3 * n));
  for (int64_t k = 0; k < n_modes; ++k)
    for (int ax = 0; ax < 3; ++ax)
      for (int64_t c = 0; c < n; ++c) {
        int64_t idx = (modes[3 * k + ax] * c) % n;
        if (idx < 0) idx += n;
        tr[(k * 3 + ax) * n + c] = cos(2.0 * M_PI * (double)idx / (double)n);
        ti[(k * 3 + ax) * n + c] = -sin(2.0 * M_PI * (double)idx / (double)n);
      }
  const int nt = omp_get_max_threads();
  double* pr = (double*)calloc((size_t)(nt * n_modes), sizeof(double));
  double* pi = (double*)calloc((size_t)(nt * n_modes), sizeof(double));
#pragma omp parallel
  {
    const int tid = omp_get_thread_num();
    /* thread-local sums (no shared cache lines while accumulating) */
    double* my_re = (double*)calloc((size_t)n_modes, sizeof(double));
    double* my_im = (double*)calloc((size_t)n_modes, sizeof(double));
    int64_t cell[3][MAXP];
    double w[3][MAXP];
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n_p; ++j) {
      for (int ax = 0; ax < 3; ++ax) stencil(u[3 * j + ax], p, n, cell[ax], w[ax]);
      for (int64_t k = 0; k < n_modes; ++k) {
        double fr = 1.0, fi = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
          const double* cr = tr + (k * 3 + ax) * n;
          const double* ci = ti + (k * 3 + ax) * n;
          double ar = 0.0, ai = 0.0;
          for (int t = 0; t < p; ++t) {
            ar += w[ax][t] * cr[cell[ax][t]];
            ai += w[ax][t] * ci[cell[ax][t]];
          }
          const double r = fr * ar - fi * ai;
          fi = fr * ai + fi * ar;
          fr = r;
        }
        my_re[k] += fr;
        my_im[k] += fi;
      }
    }
    for (int64_t k = 0; k < n_modes; ++k) {
      pr[(int64_t)tid * n_modes + k] = my_re[k];
      pi[(int64_t)tid * n_modes + k] = my_im[k];
    }
    free(my_re);
    free(my_im);
  }
  for (int64_t k = 0; k < n_modes; ++k) {
    out_re[k] = 0.0;
    out_im[k] = 0.0;
    for (int t = 0; t < nt; ++t) {
      out_re[k] += pr[(int64_t)t * n_modes + k];
      out_im[k] += pi[(int64_t)t * n_modes + k];
    }
  }
  free(pr);
  free(pi);
  free(tr);
  free(ti);
}

/* rho at k sampled cells (k x 3): sum over particles of the stencil weight
 * of each sampled cell it holds */
void oracle_cell_values(const double* u, int64_t n_p, int64_t n, int p,
                        const int64_t* cells, int64_t k, double* out) {
  const int nt = omp_get_max_threads();
  double* part = (double*)calloc((size_t)(nt * k), sizeof(double));
#pragma omp parallel
  {
    const int tid = omp_get_thread_num();
    double* mine = (double*)calloc((size_t)k, sizeof(double));
    int64_t cell[3][MAXP];
    double w[3][MAXP];
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n_p; ++j) {
      for (int ax = 0; ax < 3; ++ax) stencil(u[3 * j + ax], p, n, cell[ax], w[ax]);
      for (int64_t i = 0; i < k; ++i) {
        double prod = 1.0;
        for (int ax = 0; ax < 3 && prod != 0.0; ++ax) {
          double s = 0.0;
          for (int t = 0; t < p; ++t)
            if (cell[ax][t] == cells[3 * i + ax]) s += w[ax][t];
          prod *= s;
        }
        mine[i] += prod;
      }
    }
    for (int64_t i = 0; i < k; ++i) part[(int64_t)tid * k + i] = mine[i];
    free(mine);
  }
  for (int64_t i = 0; i < k; ++i) {
    out[i] = 0.0;
    for (int t = 0; t < nt; ++t) out[i] += part[(int64_t)t * k + i];
  }
  free(part);
}

/* shell of |m|^2: largest b with (2b-1) n_dk <= isqrt(4 m2) (0 below bin 1) */
static int64_t shell(int64_t m2, int64_t n_dk) {
  const int64_t x = 4 * m2;
  int64_t r = (int64_t)sqrt((double)x);
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return ((r / n_dk) + 1) / 2;
}

/* mode counts (weights 1 on m_z = 0 and N/2, else 2) and sum w|m| per bin */
void oracle_mode_table(int64_t n, int64_t n_dk, int64_t n_bins, int64_t* counts,
                       double* ksum) {
  for (int64_t b = 0; b < n_bins; ++b) {
    counts[b] = 0;
    ksum[b] = 0.0;
  }
  for (int64_t ix = 0; ix < n; ++ix) {
    const int64_t mx = (ix <= n / 2) ? ix : ix - n;
    for (int64_t iy = 0; iy < n; ++iy) {
      const int64_t my = (iy <= n / 2) ? iy : iy - n;
      for (int64_t mz = 0; mz <= n / 2; ++mz) {
        const int64_t m2 = mx * mx + my * my + mz * mz;
        if (m2 == 0) continue;
        const int64_t b = shell(m2, n_dk);
        if (b < 1 || b > n_bins) continue;
        const int64_t wgt = (mz == 0 || mz == n / 2) ? 1 : 2;
        counts[b - 1] += wgt;
        ksum[b - 1] += (double)wgt * sqrt((double)m2);
      }
    }
  }
}
