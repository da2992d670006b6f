/*
 * fsest.h - C ABI of the interlaced, order-p Fourier-space estimators of
 * Sefusatti, Crocce, Scoccimarro & Couchman, "Accurate Estimators of
 * Correlation Functions in Fourier Space" (arXiv:1512.07295), on one AMD
 * Instinct MI355X (gfx950).
 *
 * Pipeline (one handle = one grid size, box, order and interlacing choice,
 * for a batch of one or more particle sets that share them):
 *
 *   estimator_deposit    particles -> primary grid (and the grid shifted by
 *                        H/2 on every axis when interlacing)       Sec. 2.3, 3.1
 *   estimator_transform  3D FFT of both grids                      Sec. 2.3
 *   estimator_power      interlace, deconvolve, bin P(k)           Sec. 3.1, 2.2
 *   estimator_bispectrum FFT-shell bispectrum                      Sec. 4.1
 *   estimator_backward   dL/dx of a loss of P(k)       (adjoint, not in paper)
 *   estimator_graph_*    the deposit->transform->power sequence captured
 *                        once as a HIP graph and replayed
 *
 * Conventions (shared by every entry point):
 *   - Positions: row-major (n, 3) arrays of x, y, z in the units of `box`,
 *     float32 or float64, in device memory.  Any finite value is accepted and
 *     wrapped periodically into [0, box).  Non-finite values give unspecified
 *     (but memory-safe) results.
 *   - Grid: point g = 0..N-1 sits at x = g H, H = box/N (grid-1 origin at 0).
 *   - Fourier convention: forward transform exp(-i k.x); signed frequency of
 *     FFT index i is i for i <= N/2, i - N above (Nyquist index -> +N/2).
 *   - Normalisation: P = V |delta|^2 with delta = N_P^-1 sum_j exp(-i k.x_j)
 *     in the alias-free limit (shot noise V/N_P); B = V^2 <delta delta delta>.
 *     The paper's (2 pi)^3 factors only rescale these.
 *   - Shells: width dk = n_dk * k_f (k_f = 2 pi / box), centred on b dk,
 *     lower-inclusive, decided on integer |m|^2; b = 1..n_bins; k = 0 unused.
 *   - Every call enqueues work on the stream given to estimator_create and
 *     returns without synchronising the host; device outputs are valid once
 *     that stream reaches the point of the call.  The library owns no device
 *     memory: the caller provides a workspace of estimator_workspace_bytes()
 *     bytes that must outlive the handle.
 *   - Errors: every entry point returns an est_status; on failure
 *     estimator_last_error() (thread-local, never NULL) describes it.  All
 *     argument checks happen on the host before any launch, so they need no
 *     GPU.  After a device error the handle can still be destroyed.
 */
#ifndef FSEST_H
#define FSEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct est_ctx* est_handle;

typedef enum {
  EST_OK = 0,
  EST_EINVAL = 1,       /* invalid argument                                  */
  EST_ENOMEM = 2,       /* workspace too small / size overflow               */
  EST_ESTATE = 3,       /* call out of order (e.g. power before transform)   */
  EST_EDEVICE = 4,      /* HIP runtime or kernel launch failure              */
  EST_EUNSUPPORTED = 5  /* valid but not implemented (e.g. N = 28)            */
} est_status;

typedef enum { EST_F32 = 0, EST_F64 = 1 } est_dtype;

/* est_config.flags.  Particles are bucket-sorted (4^3-cell buckets) before
 * the deposit.  By default the sort works in two levels without
 * device-scope atomics: per-workgroup histograms over super-buckets of
 * up to 16^3 buckets (the edge is the largest divisor of N/4 up to 16),
 * then one workgroup per super-bucket.  That workgroup count
 * bounds the second level, so for strongly clustered inputs (a large
 * fraction of all particles inside one super-bucket) this flag selects
 * the single-level counting sort with device-scope atomics instead.  The
 * atomic sort is also used whenever batch times the number of super-buckets
 * exceeds 8192.  Both
 * give identical grids. */
#define EST_FLAG_ATOMIC_SORT 1
/* The handle reserves room for per-particle masses (8 bytes per particle):
 * see estimator_set_weights. */
#define EST_FLAG_WEIGHTS 2

typedef struct {
  int32_t n_grid;        /* N in [8, 1024], a multiple of 4 of the form        */
                         /* 2^a 3^b 5^c (e.g. 100, 480, 800: mixed-radix FFT); */
                         /* above 16 also N >= 15 + order                      */
  int32_t order;         /* p = 1..6: NGP, CIC, TSC, PCS (Sec. 2.3), then the  */
                         /* order-5/6 B-splines (p-fold box convolutions)      */
  int32_t interlace;     /* 0: one grid; 1: second grid shifted by H/2 on     */
                         /* every axis (Sec. 3.1, eq. intdelta); more grids    */
                         /* (Sec. 3.1 mentions them without writing them out): */
                         /* 2: four grids, shifts 0, (1,1,0), (1,0,1), (0,1,1) */
                         /* times H/2 (no alias image of mixed parity); 3: all */
                         /* eight H/2 shift combinations (no image with an odd */
                         /* component).  delta = (1/G) sum_j F_j e^{ik.s_j}.   */
                         /* Codes 2, 3 take G/2 complex grids per set.         */
  int32_t batch;         /* number of particle sets sharing the grid, >= 1    */
  double box;            /* L > 0, finite (periodic cube of side L, Sec. 2.1) */
  int64_t max_particles; /* upper bound of n_total per call, 1 .. 2^31-1      */
  int32_t flags;         /* EST_FLAG_ATOMIC_SORT | EST_FLAG_WEIGHTS (below)    */
  int32_t reserved;      /* must be 0                                          */
} est_config;

/* Bytes of device workspace a handle with this configuration needs.
 * Host only.  EINVAL for an invalid config, EUNSUPPORTED for an N outside
 * the set above, ENOMEM if the size overflows. */
est_status estimator_workspace_bytes(const est_config* cfg, size_t* bytes);

/* Create a handle.  `workspace` is a device pointer to at least
 * estimator_workspace_bytes(cfg) bytes, 256-byte aligned, owned by the caller.
 * `stream` is a hipStream_t (NULL = the default stream).  Initialises the
 * handle's tables on that stream.  ENOMEM if workspace_bytes is too small. */
est_status estimator_create(const est_config* cfg, void* workspace,
                            size_t workspace_bytes, void* stream,
                            est_handle* out);

/* Destroy a handle (frees host state and any captured graph).  Safe on NULL
 * and after errors.  Does not touch the workspace. */
est_status estimator_destroy(est_handle h);

/* Mass assignment (Sec. 2.3, eq. delgrid) onto the primary grid and, when
 * interlacing, onto the grid sampled at x + H/2 (Sec. 3.1).
 *   pos      device (n_total, 3) positions of `dtype`.
 *   offsets  device int64 [batch + 1] prefix sums (offsets[0] = 0,
 *            offsets[batch] = n_total, non-decreasing); must be NULL when
 *            batch == 1 and non-NULL otherwise.  Set i holds particles
 *            offsets[i] .. offsets[i+1]-1.  An empty set gives a zero grid.
 *   n_total  1 .. max_particles.
 * EINVAL on a bad argument.  Overwrites both grids of every set. */
est_status estimator_deposit(est_handle h, const void* pos, est_dtype dtype,
                             const int64_t* offsets, int64_t n_total);

/* Forward 3D FFT of the deposited grids (Sec. 2.3, eqs. tdelG1-tdelG2).
 * ESTATE before a deposit.  The last axis may be completed lazily by the
 * next estimator_power / estimator_bispectrum call. */
est_status estimator_transform(est_handle h);

/* Interlace (eq. intdelta), deconvolve by prod_i sinc^p (eqs.
 * windowcorrection, intkerFT) and average V|delta|^2 in |k| shells.
 *   n_dk       shell width in units of k_f, >= 1.
 *   n_bins     1 .. N/(2 n_dk) (shells up to the Nyquist frequency).
 *   subtract_shot  0 = raw P, 1 = P - V/N_P (per set).
 *   k, p       device float64 [batch][n_bins]: mean |k| and P per shell.
 *   nmodes     device int64 [batch][n_bins]: modes per shell (full grid).
 * ESTATE before estimator_transform.  A set with no particles gives NaN. */
est_status estimator_power(est_handle h, int32_t n_dk, int32_t n_bins,
                           int32_t subtract_shot, double* k, double* p,
                           int64_t* nmodes);

/* Bytes of extra device workspace estimator_bispectrum needs for shells of
 * width n_dk k_f, n_bins shells and n_tri triangles (e.g. about 11.3 GB for
 * 128 shells of 2 k_f and all 185,056 closed triangles).  Host only; EINVAL
 * under the same conditions as estimator_bispectrum. */
est_status estimator_bispectrum_workspace_bytes(est_handle h, int32_t n_dk,
                                                int32_t n_bins, int64_t n_tri,
                                                size_t* bytes);

/* FFT-shell bispectrum (Sec. 4.1, eqs. Best, VBest, Best2, IntI) of set 0
 * (or of `mock`), shells of width n_dk k_f.
 *   tri_host   host int32 [n_tri][3], 1 <= b3 <= b2 <= b1 <= n_bins; read
 *              during the call only.
 *   bws        device workspace of estimator_bispectrum_workspace_bytes().
 *   b          device float64 [n_tri]: V^2 sum III / sum JJJ (NaN if no
 *              closed triplet).
 *   ntri       device float64 [n_tri]: number of closed mode triplets.
 * The shell fields are evaluated on a grid of M points per axis, the
 * smallest 2^a 3^b 5^c above 3 R (R the largest |m_a| of the shells; M <= N):
 * like N under the triangle limit, such an M keeps every triplet sum free of
 * aliased terms, so the results are those of the N grid up to rounding.
 * The count sums (sum JJJ) do not depend on the data: the handle keeps them
 * after a call and reuses them while M, n_dk, n_bins and the triangles' tiles
 * stay the same.  Host-synchronising.
 * EINVAL if (n_bins + 1/2) n_dk >= N/3 (the triangle limit of Sec. 4.1).
 * ESTATE before estimator_transform. */
est_status estimator_bispectrum(est_handle h, int32_t mock, int32_t n_dk,
                                int32_t n_bins, const int32_t* tri_host,
                                int64_t n_tri, void* bws, size_t bws_bytes,
                                double* b, double* ntri);

/* Adjoint of deposit -> transform -> power for a loss L(P): given
 * dL/dP_b (device float64 [batch][n_bins]) writes dL/dx (device, same dtype
 * and layout as pos) for every particle.  The grids are recomputed from pos
 * (nothing is kept from the forward); the handle's grids are overwritten.
 * Same argument rules as estimator_deposit and estimator_power.  With
 * interlace codes 2 and 3 the handle holds an extra half-spectrum buffer
 * for the combined C(m) (8 bytes per mode and set). */
est_status estimator_backward(est_handle h, const void* pos, est_dtype dtype,
                              const int64_t* offsets, int64_t n_total,
                              const double* dldp, int32_t n_dk, int32_t n_bins,
                              void* grad);

/* Capture deposit -> transform -> power with these arguments into a HIP
 * graph owned by the handle (replacing any earlier one).  Pointers are baked
 * into the graph; the buffers must stay valid while it is replayed.  Also
 * runs the pipeline once. */
est_status estimator_graph_capture(est_handle h, const void* pos,
                                   est_dtype dtype, const int64_t* offsets,
                                   int64_t n_total, int32_t n_dk,
                                   int32_t n_bins, int32_t subtract_shot,
                                   double* k, double* p, int64_t* nmodes);

/* Replay the captured graph on the handle's stream.  ESTATE if none. */
est_status estimator_graph_launch(est_handle h);

/* Pick this handle's launch shapes (strided-FFT lines per workgroup, P(k)
 * reduction workgroups, deposit workgroup size, deposit work grouped per
 * XCD) by timing the whole pipeline on the given input `iters` times per
 * candidate, one parameter at a time.  The 32-bit fixed-point deposit stays
 * selected (it runs only where provably safe); estimator_set_launch can
 * force the 64-bit one.  Returns the chosen combination as an index in
 * [0, 48) in *choice.  Results do not depend on the choice beyond rounding.
 * Host-synchronising. */
est_status estimator_autotune(est_handle h, const void* pos, est_dtype dtype,
                              const int64_t* offsets, int64_t n_total,
                              int32_t n_dk, int32_t n_bins, int32_t iters,
                              int32_t* choice);

/* Set the launch shapes directly from an index returned by
 * estimator_autotune (e.g. one cached from an earlier run).  EINVAL outside
 * [0, 48).  Until a handle's shapes are set or tuned, its deposit workgroup
 * size is chosen per kernel (1024 threads where two such workgroups fit on
 * a CU, else 512). */
est_status estimator_set_launch(est_handle h, int32_t choice);

/* Per-particle masses (the paper takes equal masses for simplicity,
 * Sec. 2.1; a mass w_j weights particle j's kernel in eq. delgrid).
 * `weights` is a device array of float32 masses, w[j] for particle j in the
 * order of the positions passed to the following estimator_deposit,
 * estimator_backward, estimator_graph_capture, estimator_autotune and
 * estimator_direct_delta calls on this handle (n_total, or n, entries); NULL
 * restores equal masses.  The library keeps the pointer, not the data: the
 * array must stay valid while those calls run, and a captured graph reads
 * the array set at capture time on every launch.  With masses, delta is
 * normalised by the total mass W = sum w_j of its set, the subtracted shot
 * noise is V sum w^2 / W^2, and dL/dx_j carries the factor w_j.  Masses must
 * be finite and >= 0: a negative, NaN or infinite mass makes every grid
 * value of the call NaN (and so P(k)); all-zero masses give W = 0 and NaN
 * P(k).  Host only; EINVAL for a NULL handle or one created without
 * EST_FLAG_WEIGHTS. */
est_status estimator_set_weights(est_handle h, const float* weights);

/* Test hook: copy grid `which` (1 = primary, 2 = interlaced; up to 8 with
 * interlace codes 2, 3, in the order of their shifts) of set `mock`
 * as float32 [N][N][N] (z fastest) to dst (device).  ESTATE unless the last
 * call was estimator_deposit. */
est_status estimator_copy_grid(est_handle h, int32_t which, int32_t mock,
                               float* dst);

/* Test hook: delta(m) = C(m) / (N_P W(m)) of set `mock` at n signed integer
 * modes (device int32 [n][3], each component in (-N/2, N/2]) into device
 * float64 [n][2] (re, im).  Brings the handle to the full-spectrum state. */
est_status estimator_sample_delta(est_handle h, int32_t mock,
                                  const int32_t* modes, int64_t n,
                                  double* out);

/* ---- Direct summation and half-spectrum statistics (Sec. 2.2; Sec. 3.2,
 * comparison to direct summation).  A half spectrum is a device float64
 * array [N][N][N/2+1][2] (re, im): entry (ix, iy, m_z) holds the mode
 * (m_x, m_y, m_z) with m = ix for ix <= N/2 and ix - N otherwise (index N/2
 * is +N/2), the same for y, and m_z = 0 .. N/2. */

/* Bytes of device workspace estimator_direct_delta needs for n particles
 * (the handle's N).  Host only. */
est_status estimator_direct_workspace_bytes(est_handle h, int64_t n,
                                            size_t* bytes);

/* Alias-free Fourier density by direct summation (eq. deltaDS):
 * delta_DS(m) = n^-1 sum_j exp(-2 pi i m . x_j / L) at every mode of the
 * handle's half spectrum, for the n positions pos (device, [n][3] float32 or
 * float64, wrapped into [0, L) like the deposit), written to out (device
 * half spectrum).  dws: caller-owned device workspace of
 * estimator_direct_workspace_bytes(h, n) bytes, 256-byte aligned.  Each
 * position is reduced to 32-bit fixed-point phases (error < 2^-32 turns per
 * unit of m); terms are summed in FP32 per chunk of 256 particles and in
 * FP64 across chunks.  Cost N_P N^3 / 2 terms (ALU-bound).  Independent of
 * the handle's deposit state. */
est_status estimator_direct_delta(est_handle h, const void* pos,
                                  est_dtype dtype, int64_t n, void* dws,
                                  size_t dws_bytes, double* out);

/* estimator_direct_delta without a caller workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as estimator_direct_delta; the workspace is instead a static
 * device array of 64 MiB that the library holds on every GPU it runs on
 * until the process ends (its device address is looked up once per device
 * by estimator_create).  This call allocates nothing.  EST_ENOMEM (nothing
 * launched) when estimator_direct_workspace_bytes(h, n) exceeds 64 MiB, e.g.
 * about 4e5 particles on N = 64.  Every call on one GPU shares that array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, handles or threads) race and must be serialised by the caller;
 * calls on one stream are ordered by it. */
est_status estimator_direct_delta_noalloc(est_handle h, const void* pos,
                                          est_dtype dtype, int64_t n,
                                          double* out);

/* The estimator's delta(m) = C(m) / (N_P W(m)) (eqs. intdelta,
 * windowcorrection; normalised like the direct sum) of set `mock` at every
 * half-spectrum mode, into out (device half spectrum).  Needs
 * estimator_transform first; brings the handle to the full-spectrum state. */
est_status estimator_export_delta(est_handle h, int32_t mock, double* out);

/* Shell statistics of two half spectra a, b (device; b may be NULL for
 * b = a): P_b = V sum_{m in shell b} w Re(a(m) b*(m)) / N_b - shot, with the
 * shells, half-spectrum weights w and mode counts of estimator_power (eq. ps).
 * With a = b = delta_DS this is the direct-summation estimator of Sec. 2.2
 * (shot noise V / N_P when shot is set to it); with a = delta_G and
 * b = delta_DS the cross spectrum P_{G-DS} used to measure aliasing in
 * Sec. 3.2.  Outputs
 * k (mean |k| per shell), p, nmodes: device [n_bins]. */
est_status estimator_spectrum_power(est_handle h, const double* a,
                                    const double* b, int32_t n_dk,
                                    int32_t n_bins, double shot, double* k,
                                    double* p, int64_t* nmodes);

/* Per-kernel-group timing (tracing).  enable = 1 clears the accumulators
 * and from then on brackets every kernel group a call launches (bucket sort,
 * deposit, each FFT pass, the fused P(k) pass, ...) with HIP events on the
 * handle's stream; enable = 0 stops.  Recording is asynchronous; it is
 * skipped inside graph capture. */
est_status estimator_profile(est_handle h, int32_t enable);

/* Synchronise the handle's stream and report label `idx` (0-based): its
 * name (NUL-terminated, truncated to name_len), total milliseconds and
 * number of launches since profiling was enabled.  *n_labels receives the
 * number of labels; EINVAL if idx is out of range (after setting it). */
est_status estimator_profile_read(est_handle h, int32_t idx, char* name,
                                  size_t name_len, double* total_ms,
                                  int64_t* launches, int32_t* n_labels);

/* Message of the last failed call on this thread ("" if none). */
const char* estimator_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FSEST_H */
