// fft_reg.h -- thread-private mixed-radix FFTs of compile-time length N over
// a register array, for the transforms of the field contraction.
//
//   out[k] = sum_n in[n] exp(SIGN 2 pi i n k / N),  SIGN = -1 or +1.
//
// Decimation in time: N = R_1 R_2 ... R_S (radices 4, 2, 3, 5, in that order
// of preference).  The caller loads input n into register position
// FftPlan<N>::pos(n) (the mixed-radix digit reversal), then run() performs
// the butterfly stages in place, innermost factor first, leaving output k in
// position k.  Every loop has compile-time bounds and every twiddle is a
// compile-time constant, so the array stays in registers and no twiddle is
// loaded at run time.
#pragma once

#include <hip/hip_runtime.h>

namespace u1ml {
namespace fftreg {

// --- compile-time cos / sin of 2 pi k / n ---------------------------------
constexpr double kPi = 3.14159265358979323846;

// Taylor series, |x| <= pi / 4: 12 terms leave an error far below 1 ulp
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 12; ++i) {
    term *= -x * x / (double)((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 12; ++i) {
    term *= -x * x / (double)((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi k / n by reduction to an octant: with 8 k = o n + rem,
// the angle is o pi / 4 + 2 pi rem / (8 n), 0 <= rem < n
constexpr double cos2pi(int k, int n) {
  k %= n;
  if (k < 0) k += n;
  const int o = (8 * k) / n, rem = 8 * k - o * n;
  const double a = 2.0 * kPi * (double)rem / (8.0 * (double)n);  // [0, pi/4)
  // cos(o pi/4 + a) from cos a, sin a and the octant
  const double c = taylor_cos(a), s = taylor_sin(a), h = 0.70710678118654752440;
  switch (o) {
    case 0: return c;
    case 1: return h * (c - s);
    case 2: return -s;
    case 3: return -h * (c + s);
    case 4: return -c;
    case 5: return -h * (c - s);
    case 6: return s;
    default: return h * (c + s);
  }
}
constexpr double sin2pi(int k, int n) { return cos2pi(4 * k - n, 4 * n); }  // sin t = cos(t - pi/2)

// --- plan ------------------------------------------------------------------
template <int N>
struct FftPlan {
  static constexpr int radix_of(int m) {
    return m % 4 == 0 ? 4 : m % 2 == 0 ? 2 : m % 3 == 0 ? 3 : m % 5 == 0 ? 5 : m;
  }
  static constexpr bool supported() {
    int m = N;
    while (m > 1) {
      const int r = radix_of(m);
      if (r != 2 && r != 3 && r != 4 && r != 5) return false;
      m /= r;
    }
    return N >= 1;
  }
  // position of input n: sum_s digit_s(n) * M_s, with n = d_1 + R_1 (d_2 + R_2 (...))
  // and M_s = N / (R_1 ... R_s)
  static constexpr int pos(int n) {
    int m = N, p = 0;
    while (m > 1) {
      const int r = radix_of(m);
      m /= r;
      p += (n % r) * m;
      n /= r;
    }
    return p;
  }
};

// compile-time tables, indexed with unrolled loop counters (so every lookup
// folds to a constant)
template <int N>
struct PosTable {
  int v[N];
  constexpr PosTable() : v() {
    for (int n = 0; n < N; ++n) v[n] = FftPlan<N>::pos(n);
  }
};
template <int N>
struct TwTable {  // exp(2 pi i e / N) = (c[e], s[e])
  double c[N], s[N];
  constexpr TwTable() : c(), s() {
    for (int e = 0; e < N; ++e) {
      c[e] = cos2pi(e, N);
      s[e] = sin2pi(e, N);
    }
  }
};
template <int N>
__device__ constexpr PosTable<N> kPos{};
template <int N>
__device__ constexpr TwTable<N> kTw{};

// --- butterflies -------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// a * (c + i s)
__device__ __forceinline__ double2 cmulc(double2 a, double c, double s) {
  return make_double2(a.x * c - a.y * s, a.x * s + a.y * c);
}
// SIGN i * a
template <int SIGN>
__device__ __forceinline__ double2 rot(double2 a) {
  return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <int R, int SIGN>
struct Radix;

template <int SIGN>
struct Radix<2, SIGN> {
  static __device__ __forceinline__ void run(double2 (&a)[2]) {
    const double2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <int SIGN>
struct Radix<4, SIGN> {
  static __device__ __forceinline__ void run(double2 (&a)[4]) {
    const double2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const double2 s13 = cadd(a[1], a[3]), d13 = rot<SIGN>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
  }
};

template <int SIGN>
struct Radix<3, SIGN> {
  static __device__ __forceinline__ void run(double2 (&a)[3]) {
    constexpr double h = 0.86602540378443864676;  // sin(2 pi / 3)
    const double2 t = cadd(a[1], a[2]);
    const double2 u = rot<SIGN>(csub(a[1], a[2]));
    const double2 m = make_double2(a[0].x - 0.5 * t.x, a[0].y - 0.5 * t.y);
    a[0] = cadd(a[0], t);
    a[1] = make_double2(m.x + h * u.x, m.y + h * u.y);
    a[2] = make_double2(m.x - h * u.x, m.y - h * u.y);
  }
};

template <int SIGN>
struct Radix<5, SIGN> {
  static __device__ __forceinline__ void run(double2 (&a)[5]) {
    constexpr double c1 = cos2pi(1, 5), c2 = cos2pi(2, 5), s1 = sin2pi(1, 5), s2 = sin2pi(2, 5);
    const double2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const double2 u1 = rot<SIGN>(csub(a[1], a[4])), u2 = rot<SIGN>(csub(a[2], a[3]));
    const double2 m1 = make_double2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
    const double2 m2 = make_double2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
    const double2 n1 = make_double2(s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y);
    const double2 n2 = make_double2(s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y);
    a[0] = make_double2(a[0].x + t1.x + t2.x, a[0].y + t1.y + t2.y);
    a[1] = cadd(m1, n1);
    a[4] = csub(m1, n1);
    a[2] = cadd(m2, n2);
    a[3] = csub(m2, n2);
  }
};

// one stage: blocks of NS = R * MS positions; within each, for k1 < MS the R
// values at r MS + k1 are multiplied by exp(SIGN 2 pi i r k1 / NS) and
// transformed over r, output k2 going to k1 + MS k2
template <int N, int R, int MS, int SIGN>
__device__ __forceinline__ void stage(double2 (&y)[N]) {
  constexpr int NS = R * MS;
#pragma unroll
  for (int b = 0; b < N / NS; ++b) {
#pragma unroll
    for (int k1 = 0; k1 < MS; ++k1) {
      double2 a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double2 v = y[b * NS + r * MS + k1];
        const int e = (r * k1) % NS;
        a[r] = e == 0 ? v : cmulc(v, kTw<NS>.c[e], (double)SIGN * kTw<NS>.s[e]);
      }
      Radix<R, SIGN>::run(a);
#pragma unroll
      for (int r = 0; r < R; ++r) y[b * NS + r * MS + k1] = a[r];
    }
  }
}

// stages from the innermost factor outwards: factor s of N = R_1 ... R_S acts
// with MS = N / (R_1 ... R_s)
template <int N, int M, int SIGN>
struct Stages {
  // M: length of the transform still to be factored at this level
  static constexpr int R = FftPlan<N>::radix_of(M);
  static __device__ __forceinline__ void run(double2 (&y)[N]) {
    Stages<N, M / R, SIGN>::run(y);  // inner factors first
    stage<N, R, M / R, SIGN>(y);
  }
};
template <int N, int SIGN>
struct Stages<N, 1, SIGN> {
  static __device__ __forceinline__ void run(double2 (&)[N]) {}
};

// in-place transform of y, inputs at FftPlan<N>::pos(n), outputs in order
template <int N, int SIGN>
__device__ __forceinline__ void run(double2 (&y)[N]) {
  static_assert(FftPlan<N>::supported(), "FFT length must factor into 2, 3, 5");
  Stages<N, N, SIGN>::run(y);
}

}  // namespace fftreg
}  // namespace u1ml
