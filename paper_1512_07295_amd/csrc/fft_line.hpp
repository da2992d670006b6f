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

}  // namespace fsest
