// Device helpers shared by the kernels: complex arithmetic and the LDS FFT.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace eahp {

template <typename T> __device__ __forceinline__ cplx<T> mk(T x, T y) {
  cplx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cplx<T> cjmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// s * i * a  (s = +1 or -1)
template <typename T> __device__ __forceinline__ cplx<T> muli(cplx<T> a, T s) { return mk<T>(-s * a.y, s * a.x); }

// ------------------------------------------------------------------ buffer access
// Complex loads and stores through a raw buffer resource over [base, base +
// bytes): a 32-bit byte offset per lane, the base in scalar registers.  An
// offset at or beyond `bytes` reads zero and drops the store (the hardware's
// range check), which lets a lane skip an element without a branch.
constexpr uint32_t kBufOob = 0x7ffffff0u;
constexpr int kBufDword3 = 0x00020000;
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_buf(const cplx<T>* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cplx<T>*>(base), (short)0, (int)bytes, kBufDword3);
}
template <typename T> __device__ __forceinline__ cplx<T> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ cplx<float> buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(cplx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ cplx<double> buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(cplx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<float> v) {
  using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, cplx<double> v) {
  using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), r, (int)off, 0, 0);
}

// ------------------------------------------------------------------ small DFTs
// y_k = sum_j u_j exp(sign * 2 pi i j k / R), in place.
template <typename T, int R> struct Dft;
template <typename T> struct Dft<T, 2> {
  __device__ static void run(cplx<T>* u, T) {
    cplx<T> a = u[0], b = u[1];
    u[0] = cadd<T>(a, b);
    u[1] = csub<T>(a, b);
  }
};
template <typename T> struct Dft<T, 3> {
  __device__ static void run(cplx<T>* u, T sg) {
    const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
    cplx<T> t = cadd<T>(u[1], u[2]);
    cplx<T> m = mk<T>(u[0].x - (T)0.5 * t.x, u[0].y - (T)0.5 * t.y);
    cplx<T> d = muli<T>(csub<T>(u[1], u[2]), sg * h);
    u[0] = cadd<T>(u[0], t);
    u[1] = cadd<T>(m, d);
    u[2] = csub<T>(m, d);
  }
};
template <typename T> struct Dft<T, 4> {
  __device__ static void run(cplx<T>* u, T sg) {
    cplx<T> a = cadd<T>(u[0], u[2]), b = csub<T>(u[0], u[2]);
    cplx<T> c = cadd<T>(u[1], u[3]), d = muli<T>(csub<T>(u[1], u[3]), sg);
    u[0] = cadd<T>(a, c);
    u[2] = csub<T>(a, c);
    u[1] = cadd<T>(b, d);
    u[3] = csub<T>(b, d);
  }
};
template <typename T> struct Dft<T, 5> {
  __device__ static void run(cplx<T>* u, T sg) {
    const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5)
    const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5)
    const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
    const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
    cplx<T> a1 = cadd<T>(u[1], u[4]), b1 = csub<T>(u[1], u[4]);
    cplx<T> a2 = cadd<T>(u[2], u[3]), b2 = csub<T>(u[2], u[3]);
    cplx<T> r1 = mk<T>(u[0].x + c1 * a1.x + c2 * a2.x, u[0].y + c1 * a1.y + c2 * a2.y);
    cplx<T> r2 = mk<T>(u[0].x + c2 * a1.x + c1 * a2.x, u[0].y + c2 * a1.y + c1 * a2.y);
    cplx<T> i1 = muli<T>(mk<T>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y), sg);
    cplx<T> i2 = muli<T>(mk<T>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y), sg);
    u[0] = mk<T>(u[0].x + a1.x + a2.x, u[0].y + a1.y + a2.y);
    u[1] = cadd<T>(r1, i1);
    u[4] = csub<T>(r1, i1);
    u[2] = cadd<T>(r2, i2);
    u[3] = csub<T>(r2, i2);
  }
};

// ------------------------------------------------------------------ LDS FFT
// A set of lines stored in LDS: element (line l, position j) at l * ls + j * es.
// lfast: consecutive threads take consecutive lines (use when ls == 1).
// Line l sits at row (l0 + l) mod lwrap, which lets a transform cover a
// cyclic range of rows (l0 = 0 and lwrap beyond nlines: rows 0..nlines-1).
struct Lines {
  int N, es, nlines, ls, lfast;
  int l0 = 0, lwrap = 1 << 30;
};

// Quotient by a runtime divisor without an integer division: a float
// reciprocal gives the quotient to within one for n < 2^22, then one
// correction step (all butterfly indices here are far below that).
struct FDiv {
  int d;
  float r;
};
__device__ __forceinline__ FDiv fdiv_make(int d) { return FDiv{d, 1.0f / (float)d}; }
__device__ __forceinline__ int fdiv_q(int n, FDiv f) {
  int q = (int)((float)n * f.r);
  const int rem = n - q * f.d;
  if (rem < 0) --q;
  else if (rem >= f.d) ++q;
  return q;
}

// One self-sorting (Stockham) radix-R stage, in place: every thread loads its
// butterflies into registers, the block synchronises, then writes them back.
// Requires nlines * N / R <= MAXBF * blockDim.x (checked by the host).
template <typename T, int R, int MAXBF>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, const Lines L, int span, const cplx<T>* tw, T sg) {
  const int nb = L.N / R;
  const int total = L.nlines * nb;
  const int step = L.N / (span * R);
  const int nt = blockDim.x;
  const FDiv fl = fdiv_make(L.lfast ? L.nlines : nb), fs = fdiv_make(span);
  cplx<T> u[MAXBF][R];
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int idx = threadIdx.x + b * nt;
    if (idx < total) {
      int l, i;
      if (L.lfast) { i = fdiv_q(idx, fl); l = idx - i * L.nlines; }
      else { l = fdiv_q(idx, fl); i = idx - l * nb; }
      const int k = i - fdiv_q(i, fs) * span;
      int lr = l + L.l0;
      lr -= lr >= L.lwrap ? L.lwrap : 0;
      const cplx<T>* line = buf + lr * L.ls;
#pragma unroll
      for (int j = 0; j < R; ++j) u[b][j] = line[(i + j * nb) * L.es];
#pragma unroll
      for (int j = 1; j < R; ++j) {
        cplx<T> w = tw[j * k * step];
        w.y *= -sg;  // table holds exp(-2 pi i m / N); sg = +1 conjugates
        u[b][j] = cmul<T>(u[b][j], w);
      }
      Dft<T, R>::run(u[b], sg);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int idx = threadIdx.x + b * nt;
    if (idx < total) {
      int l, i;
      if (L.lfast) { i = fdiv_q(idx, fl); l = idx - i * L.nlines; }
      else { l = fdiv_q(idx, fl); i = idx - l * nb; }
      const int is = fdiv_q(i, fs);
      const int k = i - is * span;
      const int base = is * span * R + k;
      int lr = l + L.l0;
      lr -= lr >= L.lwrap ? L.lwrap : 0;
      cplx<T>* line = buf + lr * L.ls;
#pragma unroll
      for (int j = 0; j < R; ++j) line[(base + j * span) * L.es] = u[b][j];
    }
  }
  __syncthreads();
}

// Full transform of every line: y_k = sum_j x_j exp(sg * 2 pi i j k / N).
// MAXPTS bounds nlines * N / blockDim.x.
template <typename T, int MAXPTS>
__device__ void lds_fft(cplx<T>* buf, const Lines L, const FftPlan& P, const cplx<T>* tw, T sg) {
  for (int s = 0; s < P.nst; ++s) {
    switch (P.radix[s]) {
      case 2: fft_stage<T, 2, (MAXPTS + 1) / 2>(buf, L, P.span[s], tw, sg); break;
      case 3: fft_stage<T, 3, (MAXPTS + 2) / 3>(buf, L, P.span[s], tw, sg); break;
      case 4: fft_stage<T, 4, (MAXPTS + 3) / 4>(buf, L, P.span[s], tw, sg); break;
      case 5: fft_stage<T, 5, (MAXPTS + 4) / 5>(buf, L, P.span[s], tw, sg); break;
      default: break;
    }
  }
}

// ------------------------------------------------------------------ reductions
template <typename T> __device__ __forceinline__ T warp_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Cross-lane moves of a double by DPP (both 32-bit halves with the same control).
template <int kCtrl> __device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Value of lane l (wave-uniform l) in every lane.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over the 64 lanes of a full wave, the same value in every lane: quad
// swaps and row rotations leave each 16-lane row's sum in all its lanes, the
// four row sums are then read out and added in a fixed order.
__device__ __forceinline__ double wave_allsum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x128>(v);  // row_ror:8
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Sixteen doubles held in registers; an element picked by a wave-uniform index
// compiles to indexed register moves (no scratch, no select chains).
typedef double d16 __attribute__((ext_vector_type(16)));
typedef double d8 __attribute__((ext_vector_type(8)));

template <int kCtrl> __device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, true);
}
// (v, i) pairs: the larger v wins, ties go to the smaller i.
__device__ __forceinline__ void argmax_merge(double& v, int& i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
// Arg-max over each 16-lane row of a full wave, left in every lane of the row.
__device__ __forceinline__ void row16_argmax(double& v, int& i) {
  argmax_merge(v, i, dpp_f64<0xB1>(v), dpp_i32<0xB1>(i));
  argmax_merge(v, i, dpp_f64<0x4E>(v), dpp_i32<0x4E>(i));
  argmax_merge(v, i, dpp_f64<0x124>(v), dpp_i32<0x124>(i));
  argmax_merge(v, i, dpp_f64<0x128>(v), dpp_i32<0x128>(i));
}
// Arg-max over a full wave, the same (v, i) in every lane.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  row16_argmax(v, i);
  double bv = readlane_f64(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) argmax_merge(bv, bi, readlane_f64(v, r), __builtin_amdgcn_readlane(i, r));
  v = bv;
  i = bi;
}

// Block-wide sum (blockDim.x multiple of 64, <= 1024); result valid in thread 0.
template <typename T> __device__ __forceinline__ T block_sum(T v, T* sh /* >= 16 */) {
  v = warp_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  return r;
}

}  // namespace eahp
