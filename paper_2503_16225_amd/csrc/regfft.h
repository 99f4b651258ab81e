// Register-resident DFTs of small composite sizes (N <= 16, N a product of at
// most two of 2, 3, 4, 5), every index and twiddle a compile-time constant so
// that the operands stay in registers.
#pragma once

#include "devcommon.h"

namespace eahp {

// cos and sin of 2 pi m / N for compile-time m, N: the angle is reduced to
// [-pi/4, pi/4] by the octant symmetries (exact rational arithmetic on m/N),
// then summed as Taylor series; the truncation error is below 1e-22.
struct CTrig {
  double c, s;
};
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr CTrig ctaylor(double x) {
  double c = 1.0, s = x, tc = 1.0, ts = x;
  for (int k = 1; k < 14; ++k) {
    tc *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    ts *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    c += tc;
    s += ts;
  }
  return CTrig{c, s};
}
constexpr CTrig ctrig(int m, int N) {
  m %= N;
  if (m < 0) m += N;
  // octant o = round(8 m / N) with remainder r: angle = o pi/4 + 2 pi r / (8 N)
  const int o = (8 * m + N / 2) / N;
  const int r8 = 8 * m - o * N;  // angle - o pi/4 = 2 pi r8 / (8 N), |r8| <= N/2
  const CTrig t = ctaylor(2.0 * kPi * r8 / (8.0 * N));
  const double h = 0.70710678118654752440084436210484904;  // cos(pi/4)
  switch (o & 7) {
    case 0: return CTrig{t.c, t.s};
    case 1: return CTrig{h * (t.c - t.s), h * (t.c + t.s)};
    case 2: return CTrig{-t.s, t.c};
    case 3: return CTrig{-h * (t.c + t.s), h * (t.c - t.s)};
    case 4: return CTrig{-t.c, -t.s};
    case 5: return CTrig{-h * (t.c - t.s), -h * (t.c + t.s)};
    case 6: return CTrig{t.s, -t.c};
    default: return CTrig{h * (t.c + t.s), -h * (t.c - t.s)};
  }
}

constexpr int small_factor(int N) { return N % 4 == 0 && N != 8 ? 4 : N % 2 == 0 ? 2 : N % 3 == 0 ? 3 : N % 5 == 0 ? 5 : N; }
constexpr bool is_codelet(int N) { return N == 2 || N == 3 || N == 4 || N == 5; }

// y_k = sum_j u_j exp(sg 2 pi i j k / N), in place on u[0..N).
template <typename T, int N, bool kCodelet = is_codelet(N)>
struct RegFft;
template <typename T, int N>
struct RegFft<T, N, true> {
  __device__ static __forceinline__ void run(cplx<T>* u, T sg) { Dft<T, N>::run(u, sg); }
};
template <typename T>
struct RegFft<T, 1, false> {
  __device__ static __forceinline__ void run(cplx<T>*, T) {}
};
// N = A B: j = B ja + jb, k = ka + A kb;
// y_{ka + A kb} = sum_jb w_B^{jb kb} [w_N^{jb ka} sum_ja w_A^{ja ka} u_{B ja + jb}]
template <typename T, int N>
struct RegFft<T, N, false> {
  static constexpr int A = small_factor(N), B = N / A;
  static_assert(A * B == N && is_codelet(A) && is_codelet(B), "unsupported register DFT size");
  __device__ static __forceinline__ void run(cplx<T>* u, T sg) {
    cplx<T> z[A][B];
#pragma unroll
    for (int jb = 0; jb < B; ++jb) {
      cplx<T> v[A];
#pragma unroll
      for (int ja = 0; ja < A; ++ja) v[ja] = u[B * ja + jb];
      Dft<T, A>::run(v, sg);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) {
        if (jb * ka == 0) {
          z[ka][jb] = v[ka];
        } else {
          constexpr int n = N;
          const CTrig w = ctrig(jb * ka, n);
          z[ka][jb] = cmul<T>(v[ka], mk<T>((T)w.c, sg * (T)w.s));
        }
      }
    }
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      Dft<T, B>::run(z[ka], sg);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) u[ka + A * kb] = z[ka][kb];
    }
  }
};

}  // namespace eahp
