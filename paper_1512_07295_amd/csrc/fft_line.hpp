// Complex float helpers and the in-workgroup Stockham FFT of one line.
//
// A line of length L (power of two, 4..1024) is held by TPL = L / EPT
// threads, EPT = min(16, L) complex elements each: thread t holds elements
// t + e * TPL, e = 0..EPT-1, on entry and on exit (natural order both ways).
// Stages are radix 16 except a last radix-2/4/8 stage when log2 L is not a
// multiple of 4; butterflies run in registers, data move between stages
// through LDS.  Twiddles of the runtime stages come from a table
// tw[n] = exp(-2 pi i n / L) computed in float64 on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace fsest {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// cos and sin of 2 pi k / 16
struct Tw16 {
  static constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                  0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                                  -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                                  0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
  static constexpr float s[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                  1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                  0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                                  -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
};

// a * exp(DIR * 2 pi i K / R), DIR = -1 forward, +1 inverse; K, R compile-time.
template <int DIR, int R, int K>
__device__ __forceinline__ float2 mul_const_tw(float2 a) {
  constexpr int idx = (K * (16 / R)) & 15;
  if constexpr (idx == 0) {
    return a;
  } else if constexpr (idx == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (idx == 4) {  // exp(DIR i pi/2) = DIR i
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  } else if constexpr (idx == 12) {  // exp(DIR i 3pi/2) = -DIR i
    return DIR < 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else {
    constexpr float c = Tw16::c[idx];
    constexpr float s = DIR * Tw16::s[idx];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// In-register DFT of size R (natural order in and out), radix-2 decimation in time.
template <int R, int DIR>
struct Dft {
  __device__ __forceinline__ static void run(float2* a) {
    float2 e[R / 2], o[R / 2];
    static_for<0, R / 2>([&](auto k) {
      e[k] = a[2 * k];
      o[k] = a[2 * k + 1];
    });
    Dft<R / 2, DIR>::run(e);
    Dft<R / 2, DIR>::run(o);
    static_for<0, R / 2>([&](auto k) {
      float2 t = mul_const_tw<DIR, R, decltype(k)::value>(o[k]);
      a[k] = cadd(e[k], t);
      a[k + R / 2] = csub(e[k], t);
    });
  }
};
template <int DIR>
struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(float2*) {}
};

template <int L>
struct LinePlan {
  static constexpr int EPT = L < 16 ? L : 16;
  static constexpr int TPL = L / EPT;
};

// Radix of the stage that starts at sub-transform length NS.
template <int L, int NS>
struct StageRadix {
  static constexpr int rem = L / NS;
  static constexpr int value = rem >= 16 ? 16 : rem;
};

// LDS index of element i of a line: padded rows (ls == 1) or interleaved lines.
template <int LS>
__device__ __forceinline__ int lds_index(int i) {
  if constexpr (LS == 1) {
    return i + (i >> 4);
  } else {
    return i * LS;
  }
}

template <int L>
struct LdsLine {
  // float2 elements one padded row (LS == 1) occupies
  static constexpr int padded = L + L / 16 + 1;
};

template <int L, int DIR, int LS, int NS>
__device__ __forceinline__ void fft_stage(float2 (&v)[LinePlan<L>::EPT], int t, float2* lb,
                                          const float2* __restrict__ tw) {
  constexpr int EPT = LinePlan<L>::EPT;
  constexpr int TPL = LinePlan<L>::TPL;
  constexpr int R = StageRadix<L, NS>::value;
  constexpr int NB = EPT / R;  // butterflies per thread in this stage
  constexpr bool LAST = (NS * R == L);
  constexpr bool FIRST = (NS == 1);
  static_for<0, NB>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int j = t + i * TPL;
    const int k = j & (NS - 1);
    float2 a[R];
    static_for<0, R>([&](auto q) { a[q] = v[i + q * NB]; });
    if constexpr (!FIRST) {
      constexpr int step = L / (NS * R);
      static_for<1, R>([&](auto q) {
        float2 w = tw[(decltype(q)::value * k) * step];
        if constexpr (DIR > 0) w.y = -w.y;
        a[q] = cmul(a[q], w);
      });
    }
    Dft<R, DIR>::run(a);
    if constexpr (LAST) {
      static_for<0, R>([&](auto q) { v[i + q * NB] = a[q]; });
    } else {
      const int base = (j - k) * R + k;
      static_for<0, R>([&](auto q) { lb[lds_index<LS>(base + q * NS)] = a[q]; });
    }
  });
  if constexpr (!LAST) {
    __syncthreads();
    static_for<0, EPT>([&](auto e) { v[e] = lb[lds_index<LS>(t + e * TPL)]; });
    __syncthreads();
    fft_stage<L, DIR, LS, NS * R>(v, t, lb, tw);
  }
}

// Whole-line FFT.  Every thread of the workgroup must call it (barriers).
template <int L, int DIR, int LS>
__device__ __forceinline__ void line_fft(float2 (&v)[LinePlan<L>::EPT], int t, float2* lb,
                                         const float2* __restrict__ tw) {
  fft_stage<L, DIR, LS, 1>(v, t, lb, tw);
}

// ------------------------------------------------------- 1024 = 32 x 32 lines
// A 1024-point line held by 32 threads with 32 elements each (thread t holds
// elements t + 32 e on entry and exit): a radix-32 stage in registers, one
// exchange through LDS, a second radix-32 stage with the twiddles
// tw[q t] (q < 32).  One LDS round trip and two barriers instead of the two
// of the 16 x 16 x 4 plan.

// cos of 2 pi k / 32; sin(2 pi k / 32) = cos(2 pi (k + 24) / 32)
struct Tw32 {
  static constexpr float c[32] = {
      1.0f, 0.98078528040323044f, 0.92387953251128674f, 0.83146961230254524f,
      0.70710678118654752f, 0.55557023301960218f, 0.38268343236508977f, 0.19509032201612826f,
      0.0f, -0.19509032201612826f, -0.38268343236508977f, -0.55557023301960218f,
      -0.70710678118654752f, -0.83146961230254524f, -0.92387953251128674f, -0.98078528040323044f,
      -1.0f, -0.98078528040323044f, -0.92387953251128674f, -0.83146961230254524f,
      -0.70710678118654752f, -0.55557023301960218f, -0.38268343236508977f, -0.19509032201612826f,
      0.0f, 0.19509032201612826f, 0.38268343236508977f, 0.55557023301960218f,
      0.70710678118654752f, 0.83146961230254524f, 0.92387953251128674f, 0.98078528040323044f};
};

// a * exp(DIR * 2 pi i K / 32)
template <int DIR, int K>
__device__ __forceinline__ float2 mul_tw32(float2 a) {
  constexpr int idx = K & 31;
  if constexpr (idx % 2 == 0) {
    return mul_const_tw<DIR, 16, idx / 2>(a);
  } else {
    constexpr float c = Tw32::c[idx];
    constexpr float s = DIR * Tw32::c[(idx + 24) & 31];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// In-register 32-point DFT (natural order in and out): two 16-point DFTs of
// the even and odd elements, then radix-2 butterflies.
template <int DIR>
__device__ __forceinline__ void dft32(float2 (&a)[32]) {
  float2 e[16], o[16];
  static_for<0, 16>([&](auto k) {
    e[k] = a[2 * k];
    o[k] = a[2 * k + 1];
  });
  Dft<16, DIR>::run(e);
  Dft<16, DIR>::run(o);
  static_for<0, 16>([&](auto k) {
    const float2 t = mul_tw32<DIR, decltype(k)::value>(o[k]);
    a[k] = cadd(e[k], t);
    a[k + 16] = csub(e[k], t);
  });
}

// Whole 1024-point line, LS interleaved lines in LDS (element i at i * LS).
// Every thread of the workgroup must call it (barriers).
template <int DIR, int LS>
__device__ __forceinline__ void line_fft_1024_r32(float2 (&v)[32], int t, float2* lb,
                                                  const float2* __restrict__ tw) {
  // stage 1: sub-transforms of length 1, butterfly t reads t + 32 q and
  // writes 32 t + q
  dft32<DIR>(v);
  static_for<0, 32>([&](auto q) { lb[(32 * t + decltype(q)::value) * LS] = v[q]; });
  __syncthreads();
  static_for<0, 32>([&](auto e) { v[e] = lb[(t + 32 * decltype(e)::value) * LS]; });
  __syncthreads();
  // stage 2: sub-transforms of length 32, twiddle w^(q t), w = exp(DIR 2 pi i / 1024)
  static_for<1, 32>([&](auto q) {
    float2 w = tw[decltype(q)::value * t];
    if constexpr (DIR > 0) w.y = -w.y;
    v[q] = cmul(v[q], w);
  });
  dft32<DIR>(v);
}

// ---------------------------------------------------------------- mixed radix
// Lengths L = 2^a 3^b 5^c that are not powers of two use a plan chosen at
// run time: Stockham stages of radix 16, 8, 4, 2 (the power-of-two part,
// largest first) then 3 and 5, the line held by tpl = ceil(L / 16) threads.
// Thread t holds elements t + e * tpl (e < 16, element < L) in registers on
// entry and exit, as for the power-of-two lines; between stages the line
// lives in LDS in natural order, each thread reading the inputs of its
// butterflies (at most ceil(16 / R) of radix R), then, after a barrier,
// writing their outputs.
constexpr int kRtMaxStages = 12;
struct RtLine {
  int L;
  int tpl;
  int nst;
  int radix[kRtMaxStages];
};

// radix-3 and radix-5 DFTs, natural order, sign DIR in the exponent
template <int DIR>
__device__ __forceinline__ void dft3(float2* a) {
  constexpr float s3 = DIR * 0.86602540378443865f;  // sin(2 pi / 3)
  const float2 t1 = cadd(a[1], a[2]);
  const float2 d = csub(a[1], a[2]);
  const float2 m = make_float2(a[0].x - 0.5f * t1.x, a[0].y - 0.5f * t1.y);
  const float2 r = make_float2(-s3 * d.y, s3 * d.x);  // i s3 (a1 - a2)
  a[0] = cadd(a[0], t1);
  a[1] = cadd(m, r);
  a[2] = csub(m, r);
}

template <int DIR>
__device__ __forceinline__ void dft5(float2* a) {
  constexpr float c1 = 0.30901699437494742f;   // cos(2 pi / 5)
  constexpr float c2 = -0.80901699437494742f;  // cos(4 pi / 5)
  constexpr float s1 = DIR * 0.95105651629515357f;  // sin(2 pi / 5)
  constexpr float s2 = DIR * 0.58778525229247313f;  // sin(4 pi / 5)
  const float2 b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
  const float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
  const float2 m1 = make_float2(a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y);
  const float2 m2 = make_float2(a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y);
  // i (s1 d1 + s2 d2) and i (s2 d1 - s1 d2)
  const float2 r1 = make_float2(-(s1 * d1.y + s2 * d2.y), s1 * d1.x + s2 * d2.x);
  const float2 r2 = make_float2(-(s2 * d1.y - s1 * d2.y), s2 * d1.x - s1 * d2.x);
  a[0] = cadd(a[0], cadd(b1, b2));
  a[1] = cadd(m1, r1);
  a[4] = csub(m1, r1);
  a[2] = cadd(m2, r2);
  a[3] = csub(m2, r2);
}

template <int R, int DIR>
__device__ __forceinline__ void dft_any(float2* a) {
  if constexpr (R == 3) dft3<DIR>(a);
  else if constexpr (R == 5) dft5<DIR>(a);
  else Dft<R, DIR>::run(a);
}

// One Stockham stage of radix R over a line of length L in LDS, after
// sub-transforms of length ns: butterfly j reads elements j + q L/R, applies
// the twiddles w^(q k), k = j mod ns, w = exp(DIR 2 pi i / (ns R)), and writes
// its outputs to (j - k) R + k + q ns.
// j mod ns as j - floor(j m / 2^32) ns with m = floor((2^32 - 1) / ns) + 1
// (ns >= 2): exact for j ns < 2^32, far above these lines (j < L <= 1024)
__device__ __forceinline__ int rt_mod(int j, int ns, uint32_t m) {
  return ns > 1 ? j - (int)__umulhi((uint32_t)j, m) * ns : 0;
}

template <int R, int DIR, int LS>
__device__ __forceinline__ void rt_stage(float2* lb, int t, int tpl, int L, int ns, uint32_t nsm,
                                         const float2* __restrict__ tw) {
  constexpr int NB = (16 + R - 1) / R;
  const int nbf = L / R;
  const int step = L / (ns * R);
  float2 a[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * tpl;
    if (j < nbf) {
      const int k = rt_mod(j, ns, nsm);
#pragma unroll
      for (int q = 0; q < R; ++q) a[i][q] = lb[lds_index<LS>(j + q * nbf)];
      if (ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          float2 w = tw[q * k * step];
          if constexpr (DIR > 0) w.y = -w.y;
          a[i][q] = cmul(a[i][q], w);
        }
      }
      dft_any<R, DIR>(a[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * tpl;
    if (j < nbf) {
      const int k = rt_mod(j, ns, nsm);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) lb[lds_index<LS>(base + q * ns)] = a[i][q];
    }
  }
  __syncthreads();
}

// Whole-line FFT of a run-time plan; every thread of the workgroup calls it.
template <int DIR, int LS>
__device__ __forceinline__ void line_fft_rt(float2 (&v)[16], int t, float2* lb, const RtLine& pl,
                                            const float2* __restrict__ tw) {
  const int L = pl.L, tpl = pl.tpl;
#pragma unroll
  for (int e = 0; e < 16; ++e)
    if (t + e * tpl < L) lb[lds_index<LS>(t + e * tpl)] = v[e];
  __syncthreads();
  int ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int r = pl.radix[s];
    const uint32_t nsm = ns > 1 ? 0xFFFFFFFFu / (uint32_t)ns + 1u : 0u;
    // the thread index passes through an empty asm statement in every stage,
    // so that the compiler forms each stage's LDS addresses in that stage
    // instead of hoisting those of every radix out of the loop (which spills)
    int ts = t;
    asm volatile("" : "+v"(ts));
    switch (r) {
      case 16: rt_stage<16, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
      case 8: rt_stage<8, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
      case 4: rt_stage<4, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
      case 2: rt_stage<2, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
      case 3: rt_stage<3, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
      default: rt_stage<5, DIR, LS>(lb, ts, tpl, L, ns, nsm, tw); break;
    }
    ns *= r;
  }
  // elements past L are set to zero, not kept: their registers are then free
  // during the stages
#pragma unroll
  for (int e = 0; e < 16; ++e)
    v[e] = t + e * tpl < L ? lb[lds_index<LS>(t + e * tpl)] : make_float2(0.f, 0.f);
  __syncthreads();
}

// Plan for length L (host and device); false if L has a prime factor above 5.
__host__ __device__ inline bool make_rt_line(int L, RtLine* pl) {
  if (L < 2) return false;
  int rem = L, p2 = 1;
  while (rem % 2 == 0) { rem /= 2; p2 *= 2; }
  int nst = 0;
  int r[kRtMaxStages];
  while (p2 > 1) {
    const int q = p2 >= 16 ? 16 : p2;
    r[nst++] = q;
    p2 /= q;
  }
  while (rem % 3 == 0) { rem /= 3; r[nst++] = 3; }
  while (rem % 5 == 0) { rem /= 5; r[nst++] = 5; }
  if (rem != 1 || nst > kRtMaxStages) return false;
  pl->L = L;
  pl->tpl = (L + 15) / 16;
  pl->nst = nst;
  for (int i = 0; i < kRtMaxStages; ++i) pl->radix[i] = i < nst ? r[i] : 1;
  return true;
}

}  // namespace fsest
