// Mass assignment (Sec. 2.3, eq. delgrid) onto the primary grid and the grids
// shifted by half a cell (Sec. 3.1).
//
// Design (gfx950): the particles arrive sorted by bucket (sort.hip), so every
// deposit workgroup owns one output tile of T^3 cells outright: it reads the
// particles of the buckets that can reach the tile, adds the clipped
// footprints of two grids with LDS integer atomics on a fixed-point format,
// and writes the finished tile once with coalesced stores.  No global atomics
// touch the grid and the grid needs no clearing.
#include <type_traits>

#include "particles.hpp"

namespace fsest {

// ------------------------------------------------------------------ deposit
// Fixed-point accumulation.  LDS float atomics are ~20x slower than integer
// ones on gfx950, so a workgroup sums its tile in unsigned integers: a weight
// product w in [0, 1] adds floor(w * S + 1/2).  Two formats:
//  * wide (64-bit): S = 2^32 - 2^8; a grid sums to N_P < 2^31 units, so no
//    cell can overflow;
//  * narrow (32-bit): S = 2^F with F chosen on the device from the largest
//    bucket count M of this deposit.  A cell only receives particles whose
//    first grid's first stencil cell lies within p + 1 cells of it per axis
//    (at most 2 buckets per axis for p <= 4, 3 for p = 5, 6), and one
//    particle gives a cell at most w_max^3 (w_max the largest 1D weight of
//    the order: 1, 1, 3/4, 2/3, 115/192, 11/20), so its sum is at most
//    K (w_max^3 S + 1/2) units with K = 8 M (27 M) possible contributors; F
//    is the largest value keeping that below 2^32.  F >= 22 is required
//    (24 with masses, where the unit is the largest mass), or the wide
//    kernel runs instead (both are launched; the one not selected returns
//    at once).  Each contribution is rounded to 2^-(F+1) <= 2^-23 of a unit
//    mass; F < 24 only happens when the largest bucket (64 cells) holds more
//    than 32 (NGP) to 108 (PCS) particles, where cells sum several units and
//    float32 accumulation would round each addition at least as coarsely.
// Integer sums are exact, so deposits are bitwise reproducible.
constexpr float kFixWide = 4294967040.0f;  // 2^32 - 2^8
constexpr int kNarrowMinBits = 22;

// The base cells of the particles that reach one cell span p + 1 cells per
// axis (both grids), so they meet at most 2 buckets per axis for p <= 4 and
// 3 for p = 5, 6.
template <int P>
__device__ __forceinline__ int narrow_bits(uint32_t maxcount) {
  // w_max^3 of the order, with a margin for the float32 rounding of the
  // weight products
  constexpr double wmax = P <= 2 ? 1.0 : (P == 3 ? 0.75 : (P == 4 ? 2.0 / 3.0 : (P == 5 ? 115.0 / 192.0 : 0.55)));
  constexpr double w3 = wmax * wmax * wmax * (1.0 + 1e-6);
  const double k = (P <= 4 ? 8.0 : 27.0) * (double)(maxcount > 0 ? maxcount : 1);
  int f = 0;
  while (f < 31 && k * (w3 * ldexp(1.0, f + 1) + 0.5) < 4294967295.0) ++f;
  return f;
}

// The 32-bit format's fraction bits for this deposit, once per deposit.
template <int P>
__global__ void k_narrow(uint32_t* stats) {
  if (threadIdx.x == 0 && blockIdx.x == 0) stats[6] = (uint32_t)narrow_bits<P>(stats[0]);
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
static_assert(kItemCap >= 2 * 1024, "an empty list holds a whole round of items (two grids)");
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
    // ((r + P - 1) mod N) - (P - 1): the same map in three operations
    return ((r + (P - 1)) & (n - 1)) - (P - 1);
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

// Adds one grid's footprint of one particle (its record, particles.hpp) to
// the tile.  Grid gi is sampled at u + 1/2 on the axes whose bit is set in
// its mask mk: there the first cell moves by the record's step and the
// offset by -/+ 1/2.
template <int P, typename AT, int WRAP, int IL>
__device__ __forceinline__ void deposit_item(uint4 rec, int gi, const Geom& g, int t0x, int t0y,
                                             int t0z, AT* sm, float scale, int mk) {
  const int n = g.n;
  constexpr int off = (P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2;
  const int sx = (int)((rec.x >> 30) & 1u), sy = (int)(rec.x >> 31), sz = (int)((rec.y >> 24) & 1u);
  // the interlaced pair's second grid is shifted on all three axes
  const bool hx = IL == 1 ? gi != 0 : (mk & 1) != 0;
  const bool hy = IL == 1 ? gi != 0 : (mk & 2) != 0;
  const bool hz = IL == 1 ? gi != 0 : (mk & 4) != 0;
  float wx[P], wy[P], wz[P];
  weights_from_offset<P>(record_offset<P>(rec.y, sx, hx), wx);
  weights_from_offset<P>(record_offset<P>(rec.z, sy, hy), wy);
  weights_from_offset<P>(record_offset<P>(rec.w, sz, hz), wz);
#pragma unroll
  for (int i = 0; i < P; ++i) wx[i] *= scale;
  const int fx = (int)(rec.x & 1023u) - off + (hx ? sx : 0);
  const int fy = (int)((rec.x >> 10) & 1023u) - off + (hy ? sy : 0);
  const int fz = (int)((rec.x >> 20) & 1023u) - off + (hz ? sz : 0);
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

// Segment of each lane's candidate `item` (the wave's candidates are c0 ..
// c0 + 63): the last t < nr with pref[t] <= item, i.e. the number of
// starts pref[0..nr] at or below it, minus one (pref[nr] = total lies above
// every candidate; empty pieces repeat a start and count twice, which
// still lands on the non-empty piece).  Lane t holds starts t and t + 64:
// one ballot counts those at or below c0 for the whole wave, and the few
// inside the window are added lane by lane.
__device__ __forceinline__ int find_segment(const DepRanges& rg, int nr, uint32_t c0,
                                            uint32_t item, int lane) {
  const uint32_t pa = lane <= nr ? rg.pref[lane] : 0xFFFFFFFFu;
  const uint32_t pb = lane + 64 <= nr ? rg.pref[lane + 64] : 0xFFFFFFFFu;
  int cnt = __popcll(__ballot(pa <= c0)) + __popcll(__ballot(pb <= c0));
  unsigned long long ia = __ballot(pa > c0 && pa <= c0 + 63);
  unsigned long long ib = __ballot(pb > c0 && pb <= c0 + 63);
  while (ia) {
    const int t = __builtin_ctzll(ia);
    cnt += item >= (uint32_t)__builtin_amdgcn_readlane((int)pa, t) ? 1 : 0;
    ia &= ia - 1;
  }
  while (ib) {
    const int t = __builtin_ctzll(ib);
    cnt += item >= (uint32_t)__builtin_amdgcn_readlane((int)pb, t) ? 1 : 0;
    ib &= ib - 1;
  }
  return cnt - 1;
}

// One workgroup owns one T^3 output tile (T = min(kTileMax, N)) of every
// grid at a time.  Per tile: (1) the particles of the buckets that can
// reach the tile are scanned in rounds of blockDim items; each grid whose
// stencil reaches the tile becomes a work item in an LDS list and counts
// towards its bank class; (2) before a round whose items would overflow the
// list, and after the last round, the list is counting-sorted by class and
// deposited with LDS integer atomics, lane l of
// virtual wave r taking sorted item r + l * W (W = virtual waves in the
// flush); (3) the finished tile is scaled back to float and written once.
//
// Work units.  `walk` (tiles smaller than the grid, N >= T + 4 kLow): a unit
// is a segment of up to seg_len consecutive tiles of one z column, taken in
// order.  A particle's items go to the tile that holds its first z cell
// f_z, whole in z: the cells they give above the tile (at most P) stay in
// the LDS rows' upper halo and move down to the next tile's first cells
// (the carry).  The segment's first tile also takes the kLow buckets below
// it, whose stencils reach into it from below (their cells below the tile
// fall into the rows' lower margin and are dropped), and the carry of its
// last tile is dropped: the next segment takes those particles again.  So a
// particle is scanned by the tiles of one z position (plus a first tile's
// look-back) and its z stencil is never split.  Otherwise a unit is one
// tile, which scans T/4 + kLow buckets per axis and keeps the items whose
// stencil reaches it.
// Workgroups loop over units b, b + gridDim, ... (a persistent grid of a few
// workgroups per CU, so the per-workgroup set-up is paid once per many
// units); `dynamic`: units are taken from a global counter (stats[1],
// zeroed with the sort) instead.  `xcd`: runs of consecutive units go to
// the same XCD (workgroup b runs on XCD b mod 8), so the buckets that
// neighbouring columns share are read through one L2.
// WT: per-particle masses (sw, bucket order, divided by the largest mass);
// a separate instantiation so that the equal-mass kernel keeps its registers
// IL: 0 one grid; 1 the interlaced pair (masks 0 and 7); 2 a pair of grids
// with run-time masks (mask_a, mask_b) written to slab q of each set
// CAP: registers capped at 64 (8 waves per SIMD) so that two 1024-thread
// workgroups share a CU (two_groups_per_cu)
template <int P, int IL, bool WIDE, int WRAP, bool WT, bool CAP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(CAP ? 8 : 1))) void k_deposit(const uint4* __restrict__ recs,
                                                  const uint32_t* __restrict__ boff,
                                                  const uint32_t* __restrict__ bcnt, float* grid,
                                                  Geom g, uint32_t* __restrict__ stats,
                                                  int exclusive, int dynamic, int xcd,
                                                  const float* __restrict__ sw, int q, int mask_a,
                                                  int mask_b, int walk, int seg_len) {
  using AT = typename std::conditional<WIDE, unsigned long long, unsigned>::type;
  constexpr int NG = IL ? 2 : 1;
  constexpr int kWords = acc_first_word<AT>() + NG * kGridWords * (int)(sizeof(AT) / 4);
  __shared__ __align__(16) uint32_t smem[kWords];
  __shared__ DepRanges rg;
  __shared__ int round_cnt[3];
  __shared__ int cls_cnt[64];
  __shared__ int cls_cur[64];
  __shared__ int next_tile;
  uint32_t* item_j = smem;
  uint8_t* item_meta = reinterpret_cast<uint8_t*>(smem + kItemCap);
  uint16_t* item_order = reinterpret_cast<uint16_t*>(smem + kItemCap + kItemCap / 4);
  AT* sm = reinterpret_cast<AT*>(smem);
  const int acc0 = acc_first_word<AT>() * 4 / (int)sizeof(AT);

  // fixed-point format for this deposit (uniform over the grid; k_narrow
  // computed it from the sort's largest bucket count)
  const int nbits = (int)stats[6];
  // with masses the step is relative to the largest mass: F >= 24 there
  constexpr int kMinBits = WT ? 24 : kNarrowMinBits;
  if (!WIDE && nbits < kMinBits) return;                // the wide kernel does it
  if (WIDE && !exclusive && nbits >= kMinBits) return;  // the narrow one does it
  const float scale = WIDE ? kFixWide : ldexpf(1.0f, nbits);
  const double inv_scale = 1.0 / (double)scale;
  // masses: items carry w / w_max (in [0, 1], so the bounds above hold) and
  // the tile is multiplied back by w_max; an invalid mass makes it NaN
  float wmul = 1.0f;
  if constexpr (WT) wmul = stats[5] ? __builtin_nanf("") : __uint_as_float(stats[4]);

  const int n = g.n, T = g.tile, nb = g.nb;
  const int tpa = (n + T - 1) / T;  // tiles per axis; the last one is ragged when T does not divide N
  const int slen = walk ? seg_len : 1;
  const int upc = (tpa + slen - 1) / slen;  // units per z column
  // (the host keeps the unit count below 2^31)
  const uint32_t units_per_set = (uint32_t)(tpa * tpa * upc);
  const uint32_t nunits = (uint32_t)g.batch * units_per_set;
  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // workgroup b runs on XCD b mod 8: with xcd, the units are dealt to the
  // XCDs in chunks of kXcdChunk consecutive units (XCD x takes chunks x,
  // x + 8, ...), each XCD's workgroups taking its units in order (gridDim a
  // multiple of 8); chunks rather than eighths, so that sets of very
  // different sizes in a batch still spread over all XCDs
  constexpr uint32_t kXcdChunk = 16;
  const bool remap =
      xcd && !dynamic && (gridDim.x & 7) == 0 && (nunits % (8 * kXcdChunk)) == 0;
  // buckets below a tile whose particles can reach it (see the ranges below)
  constexpr int kLow = (P - 1 + (IL ? 1 : 0) + kBucket - 1) / kBucket;

  uint32_t b = blockIdx.x;
  if (dynamic) {
    if (threadIdx.x == 0) next_tile = (int)atomicAdd(&stats[1], 1u);
    __syncthreads();
    b = (uint32_t)next_tile;
  }
  while (b < nunits) {
    const uint32_t li = b >> 3;  // the unit's index among its XCD's units
    const uint32_t uid =
        remap ? ((li / kXcdChunk) * 8 + (b & 7)) * kXcdChunk + li % kXcdChunk : b;
    const int mock = (int)(uid / units_per_set);
    const int urem = (int)(uid % units_per_set);
    const int tx = urem / (tpa * upc), ty = (urem / upc) % tpa, sg = urem % upc;
    const int tz1 = min(tpa, (sg + 1) * slen);
    for (int tz = sg * slen; tz < tz1; ++tz) {
      const bool first = tz == sg * slen;
      const int t0x = tx * T, t0y = ty * T, t0z = tz * T;
      // cells of this tile per axis (a multiple of kBucket)
      const int ex = min(T, n - t0x), ey = min(T, n - t0y), ez = min(T, n - t0z);

      if (threadIdx.x < 64) cls_cnt[threadIdx.x] = 0;
      if (threadIdx.x < 3) round_cnt[threadIdx.x] = 0;

      // bucket neighbourhood: particles are bucketed by their first grid's
      // first stencil cell f, and a stencil of either grid reaches the tile
      // iff f lies in [t0 - (P - 1) - S, t0 + T - 1] (S = 1 with a shifted
      // grid), i.e. in the T/4 + kLow buckets from t0/4 - kLow; or every
      // bucket.  Walking in z: the tile's own ez/4 buckets, and the kLow below
      // them for a segment's first tile.
      int cnt = T / kBucket + kLow;
      if (cnt > nb) cnt = nb;
      const int b0x = (cnt == nb) ? 0 : (t0x / kBucket - kLow + nb) % nb;
      const int b0y = (cnt == nb) ? 0 : (t0y / kBucket - kLow + nb) % nb;
      const int zlow = walk ? (first ? kLow : 0) : kLow;
      int cntz = walk ? ez / kBucket + zlow : cnt;
      if (cntz > nb) cntz = nb;
      const int b0z = (!walk && cntz == nb) ? 0 : (t0z / kBucket - zlow + nb) % nb;
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
          const int z1 = b0z + cntz;                      // exclusive end, may pass nb
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
      // the other waves clear the tile, or move the carry down, while wave 0
      // waits for the offsets
      if (first) {
        uint4* z4 = reinterpret_cast<uint4*>(smem + acc_first_word<AT>());
        constexpr int kZero4 = (kWords - acc_first_word<AT>()) / 4;
        for (int i = threadIdx.x; i < kZero4; i += nthreads) z4[i] = make_uint4(0u, 0u, 0u, 0u);
      } else {
        // every row moves down by T elements (the previous tile was whole):
        // the upper halo becomes the first cells, the rest is cleared (the
        // lower margin receives old owned cells, which are never read)
        constexpr int kRow4 = kRow * (int)sizeof(AT) / 16;
        constexpr int kShift4 = kTileMax * (int)sizeof(AT) / 16;
        static_assert(kRow * sizeof(AT) % 16 == 0 && kPlane * sizeof(AT) % 16 == 0,
                      "rows of uint4");
        for (int r = threadIdx.x; r < NG * kTileMax * kTileMax; r += nthreads) {
          const int gi = r / (kTileMax * kTileMax);
          const int lx = (r / kTileMax) % kTileMax, ly = r % kTileMax;
          uint4* row =
              reinterpret_cast<uint4*>(sm + acc0 + gi * kGridWords + lx * kPlane + ly * kRow);
          uint4 v[kRow4 - kShift4];
#pragma unroll
          for (int c = 0; c < kRow4 - kShift4; ++c) v[c] = row[kShift4 + c];
#pragma unroll
          for (int c = 0; c < kRow4; ++c)
            row[c] = c < kRow4 - kShift4 ? v[c] : make_uint4(0u, 0u, 0u, 0u);
        }
      }
      __syncthreads();
      const uint32_t total = rg.pref[rg.count];
      const int nr = rg.count;

      // Sorts the m listed items by bank class and deposits them; every
      // thread calls it with the same m, and it ends with a barrier.
      auto deposit_list = [&](int m) __attribute__((always_inline)) {
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
        // lane l of virtual wave r takes item r + l W; each item's record is
        // loaded one iteration ahead
        const int W = (m + 63) >> 6;
        const int vend = 64 * W;
        int e_cur = -1;
        uint4 rc = make_uint4(0u, 0u, 0u, 0u);
        {
          const int v = threadIdx.x;
          const int p = (v >> 6) + (v & 63) * W;
          if (v < vend && p < m) {
            e_cur = item_order[p];
            rc = recs[item_j[e_cur]];
          }
        }
        for (int v = threadIdx.x; v < vend; v += nthreads) {
          const int vn = v + nthreads;
          const int pn = (vn >> 6) + (vn & 63) * W;
          int e_nxt = -1;
          uint4 rn = make_uint4(0u, 0u, 0u, 0u);
          if (vn < vend && pn < m) {
            e_nxt = item_order[pn];
            rn = recs[item_j[e_nxt]];
          }
          if (e_cur >= 0) {
            float sc = scale;
            if constexpr (WT) sc *= sw[item_j[e_cur]];
            const int gi = item_meta[e_cur] >> 6;
            const int mk = (IL == 2) ? (gi ? mask_b : mask_a) : (gi ? 7 : 0);
            deposit_item<P, AT, WRAP, IL>(rc, gi, g, t0x, t0y, t0z, sm, sc, mk);
          }
          e_cur = e_nxt;
          rc = rn;
        }
        __syncthreads();
      };
      int fill = 0;  // items in the list (the same value in every thread)
      int rpar = 0;  // which of the three round counters this round uses

      // rounds of blockDim candidates; the cell records of kPre rounds are
      // loaded together so that their latencies overlap (one round where the
      // registers are capped: the other workgroup on the CU covers the wait)
      constexpr int kPre = CAP ? 1 : 4;
      constexpr int off = (P % 2 == 0) ? (P / 2 - 1) : (P - 1) / 2;
      for (uint32_t rb = 0; rb < total; rb += kPre * nthreads) {
        uint32_t jj[kPre];
        uint2 rec[kPre];
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
          const uint32_t r0 = rb + q * nthreads;
          const uint32_t item = r0 + threadIdx.x;
          jj[q] = 0;
          rec[q] = make_uint2(0u, 0u);
          if (r0 < total) {
            const int seg = find_segment(rg, nr, r0 + (uint32_t)(wave * 64), item, lane);
            if (item < total) {
              jj[q] = rg.start[seg] + (item - rg.pref[seg]);
              // cells and steps: the record's x word and the y word's step bit
              rec[q] = *reinterpret_cast<const uint2*>(recs + jj[q]);
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
            const uint2 r = rec[0];
            const int cx = (int)(r.x & 1023u) - off;
            const int cy = (int)((r.x >> 10) & 1023u) - off;
            const int cz = (int)((r.x >> 20) & 1023u) - off;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
              const int mk = (IL == 2) ? (gi ? mask_b : mask_a) : (gi ? 7 : 0);
              const int sx = (mk & 1) ? (int)((r.x >> 30) & 1u) : 0;
              const int sy = (mk & 2) ? (int)(r.x >> 31) : 0;
              const int sz = (mk & 4) ? (int)((r.y >> 24) & 1u) : 0;
              const int rx = rel_first<P, WRAP>(cx + sx, t0x, n);
              const int ry = rel_first<P, WRAP>(cy + sy, t0y, n);
              const int rz = rel_first<P, WRAP>(cz + sz, t0z, n);
              if (walk) {
                // own buckets: always (the cells above the tile are carried);
                // the look-back buckets: if the stencil reaches the tile, i.e.
                // starts in [-(P - 1), 0] (rel_first maps the others above T)
                int dz = cz - t0z;
                dz = dz < 0 ? dz + n : dz;
                ok[gi] = rx < kTileMax && ry < kTileMax && (dz < ez || rz <= 0);
              } else {
                ok[gi] = reaches_tile<P, WRAP>(rx, ry, rz);
              }
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
          // each wave reserves its slice of this round's items (slices in any
          // order: the integer sums do not depend on it)
          int before = 0;
          if (lane == 0) before = atomicAdd(&round_cnt[rpar], mine);
          before = __builtin_amdgcn_readfirstlane(before);
          // three counters in turn: the next round's was last read before
          // the previous round's last barrier and is next used after this
          // round's
          if (threadIdx.x == 0) round_cnt[rpar == 2 ? 0 : rpar + 1] = 0;
          auto insert = [&](int pos) __attribute__((always_inline)) {
            const unsigned long long below = (1ull << lane) - 1ull;
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
          };
          int tot;
          if (fill == 0) {
            // an empty list holds any round (at most NG x blockDim items):
            // insert at once, learn the round's total after the barrier
            insert(before);
            __syncthreads();
            tot = round_cnt[rpar];
          } else {
            __syncthreads();
            tot = round_cnt[rpar];
            // (2) the list is deposited first if this round's items would not fit
            if (fill + tot > kItemCap) {
              deposit_list(fill);
              fill = 0;
            }
            insert(fill + before);
            __syncthreads();
          }
          rpar = rpar == 2 ? 0 : rpar + 1;
          fill += tot;
          if (r0 + nthreads >= total) {  // the last round: deposit what is left
            deposit_list(fill);
            fill = 0;
          }
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
      __syncthreads();  // the tile is written before it is cleared or moved
    }
    if (dynamic) {
      if (threadIdx.x == 0) next_tile = (int)atomicAdd(&stats[1], 1u);
      __syncthreads();
      b = (uint32_t)next_tile;
    } else {
      b += gridDim.x;
    }
  }
}

// A workgroup waits at a barrier several times per tile, and with one
// workgroup per CU the whole CU waits with it.  The 32-bit pair kernel's LDS
// (74.9 KB) leaves room for two workgroups per CU; those of 1024 threads need
// 8 waves per SIMD, i.e. at most 64 VGPRs.  The instantiations listed here
// fit in 64 without scratch (the others spill and keep their registers):
// the interlaced pair, float32 positions, equal masses, orders 1 and 2, and
// order 4 with a tile smaller than the grid.  Measured at 1024^3 with 2^27
// particles (PCS): 11.8 ms with two 512-thread workgroups per CU, 10.8 ms
// with two of 1024.
template <int P, int IL, bool WIDE, int WRAP, bool WT>
__host__ __device__ constexpr bool two_groups_per_cu() {
  return !WIDE && IL == 1 && !WT && (P <= 2 || (P == 4 && WRAP != kPeriodic));
}

// threads: 256, 512 or 1024 per deposit workgroup, or 0 for the kernel's
// own choice (1024 where two_groups_per_cu, else 512)
// Segment length of the z walk: the longest of 8, 4, 2 tiles that still
// gives every workgroup of the persistent grid about 8 units (the units of a
// batch of uneven sets differ in cost).
static int walk_segment(const Geom& g, int cus) {
  const int tpa = (g.n + g.tile - 1) / g.tile;
  const int64_t cols = (int64_t)g.batch * tpa * tpa;
  int len = 8;
  while (len > 2 && cols * ((tpa + len - 1) / len) < (int64_t)cus * 64) len /= 2;
  return len;
}

template <int P, int IL, int WRAP, bool WT>
static void deposit_launch(const Geom& g, const Buffers& b, int threads, bool narrow, bool xcd,
                           int cus, const float* sw, int q, int ma, int mb, hipStream_t s) {
  const int tpa = (g.n + g.tile - 1) / g.tile;
  // the z walk needs a tile smaller than the grid and the look-back buckets
  // of a segment's first tile distinct from its own
  constexpr int kLow = (P - 1 + (IL ? 1 : 0) + kBucket - 1) / kBucket;
  const bool walk = WRAP != kPeriodic && g.n >= g.tile + kBucket * kLow;
  const int seg = walk ? walk_segment(g, cus) : 1;
  const int64_t nunits = (int64_t)g.batch * tpa * tpa * ((tpa + seg - 1) / seg);
  constexpr bool kTwo = two_groups_per_cu<P, IL, false, WRAP, WT>();
  if (narrow) {
    const int tn = threads ? threads : (kTwo ? 1024 : 512);
    // a persistent grid: 8 workgroups per CU (a multiple of 8 for the XCD
    // grouping), each looping over units
    const int64_t cap = (int64_t)cus * 8;
    const unsigned nwg = (unsigned)(nunits < cap ? nunits : cap);
    bool capped = false;
    if constexpr (kTwo) {
      if (tn == 1024) {
        hipLaunchKernelGGL((k_deposit<P, IL, false, WRAP, WT, true>), dim3(nwg), dim3(tn), 0, s,
                           (const uint4*)b.recs, b.boff, b.bcnt, (float*)b.grid, g, b.stats, 0, 0,
                           xcd ? 1 : 0, sw, q, ma, mb, walk ? 1 : 0, seg);
        capped = true;
      }
    }
    if (!capped)
      hipLaunchKernelGGL((k_deposit<P, IL, false, WRAP, WT, false>), dim3(nwg), dim3(tn), 0, s,
                         (const uint4*)b.recs, b.boff, b.bcnt, (float*)b.grid, g, b.stats, 0, 0,
                         xcd ? 1 : 0, sw, q, ma, mb, walk ? 1 : 0, seg);
  }
  // the 64-bit kernel holds one workgroup per CU; it takes units from a
  // counter, so when the 32-bit kernel does the work it costs one short wave
  // per workgroup
  const unsigned wblocks = (unsigned)(nunits < 1024 ? nunits : 1024);
  hipLaunchKernelGGL((k_deposit<P, IL, true, WRAP, WT, false>), dim3(wblocks),
                     dim3(threads ? threads : 512), 0, s, (const uint4*)b.recs, b.boff, b.bcnt,
                     (float*)b.grid, g, b.stats, narrow ? 0 : 1, 1, 0, sw, q, ma, mb,
                     walk ? 1 : 0, seg);
}

template <int P, int IL, int WRAP>
static void dispatch_deposit_w(const Geom& g, const Buffers& b, int threads, bool narrow, bool xcd,
                               int cus, const float* sw, int q, int ma, int mb, hipStream_t s) {
  if (sw) deposit_launch<P, IL, WRAP, true>(g, b, threads, narrow, xcd, cus, sw, q, ma, mb, s);
  else deposit_launch<P, IL, WRAP, false>(g, b, threads, narrow, xcd, cus, nullptr, q, ma, mb, s);
}

template <int P, int IL>
static void dispatch_deposit_t(const Geom& g, const Buffers& b, const Tune& tu, int threads,
                               const float* sw, int q, int ma, int mb, hipStream_t s) {
  const bool narrow = tu.dep_narrow != 0;
  const bool xcd = tu.dep_xcd != 0;
  if (g.tile == g.n)
    dispatch_deposit_w<P, IL, kPeriodic>(g, b, threads, narrow, xcd, tu.cus, sw, q, ma, mb, s);
  else if ((g.n & (g.n - 1)) == 0)
    dispatch_deposit_w<P, IL, kMasked>(g, b, threads, narrow, xcd, tu.cus, sw, q, ma, mb, s);
  else
    dispatch_deposit_w<P, IL, kGeneral>(g, b, threads, narrow, xcd, tu.cus, sw, q, ma, mb, s);
}

template <int P>
static void dispatch_deposit_p(const Geom& g, const Buffers& b, const Tune& tu, int threads,
                               const float* sw, hipStream_t s) {
  hipLaunchKernelGGL(k_narrow<P>, dim3(1), dim3(64), 0, s, b.stats);
  if (g.code == 0) {
    dispatch_deposit_t<P, 0>(g, b, tu, threads, sw, 0, 0, 0, s);
  } else if (g.code == 1) {
    dispatch_deposit_t<P, 1>(g, b, tu, threads, sw, 0, 0, 7, s);
  } else {
    // one pass per slab; the 64-bit kernel's tile counter restarts each time
    for (int q = 0; q < g.npair; ++q) {
      if (q > 0) (void)launch_fill_u32(b.stats + 1, 1, 0u, s);  // reported by launch_deposit
      dispatch_deposit_t<P, 2>(g, b, tu, threads, sw, q, grid_mask(g.code, 2 * q),
                               grid_mask(g.code, 2 * q + 1), s);
    }
  }
}

hipError_t launch_deposit(const Geom& g, const Buffers& b, const Tune& tu, bool weighted,
                          hipStream_t s) {
  int threads = tu.dep_threads;
  if (threads != 256 && threads != 512 && threads != 1024) threads = 0;  // per kernel
  const float* sw = weighted ? b.sw : nullptr;
  switch (g.order) {
    case 1: dispatch_deposit_p<1>(g, b, tu, threads, sw, s); break;
    case 2: dispatch_deposit_p<2>(g, b, tu, threads, sw, s); break;
    case 3: dispatch_deposit_p<3>(g, b, tu, threads, sw, s); break;
    case 4: dispatch_deposit_p<4>(g, b, tu, threads, sw, s); break;
    case 5: dispatch_deposit_p<5>(g, b, tu, threads, sw, s); break;
    default: dispatch_deposit_p<6>(g, b, tu, threads, sw, s); break;
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

}  // namespace fsest
