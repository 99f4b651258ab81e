// Complex block products on the matrix cores (v_mfma_*_16x16x4 in FP64 and
// FP32).  A complex product is four real ones on split real/imaginary planes:
//   A^H B : Re += ar br + ai bi,  Im += ar bi - ai br
//   A  M  : Re += ar mr - ai mi,  Im += ar mi + ai mr
// Operand layout of the 16x16x4 instructions (measured on gfx950): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; result slot s of lane l is
// element (4 s + l / 16, l % 16) in FP64 and (4 (l / 16) + s, l % 16) in FP32.
//
// gemm_hn (Gram matrices, Lambda, projector coefficients): the row dimension
// n is split over work-groups, each computes output tiles over its rows and
// writes the raw fragments; a second kernel sums the splits in a fixed order
// (deterministic).
// gemm_nn (frame times small matrix): one output tile per work-group, the
// inner dimension streamed through LDS 16 at a time, the tile staged through
// LDS for coalesced stores.
// Both come in several tile shapes with identical results (see below).
#include <atomic>
#include <functional>
#include <string>
#include <vector>

#include "devcommon.h"
#include "kernels.h"
#include "ops.h"

namespace eahp {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc = d4v;
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int s) { return 4 * s + (l >> 4); }
};
template <>
struct Mfma<float> {
  using acc = f4v;
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int s) { return 4 * (l >> 4) + s; }
};

// Tile shapes.  A work-group of four waves computes a TR x TC output tile,
// TR = WR BU 16 and TC = WC BV 16: the waves form a WR x WC grid and each
// holds BU x BV blocks of 16 x 16 (real and imaginary accumulators).  Every
// shape accumulates each output element over the inner dimension in the same
// order (chunks of 16 from the start of its row range, four per MFMA), so the
// shapes give identical results and differ only in speed; the autotuner picks
// one per shape class.
constexpr int kXcds = 8;     // MI355X: 8 accelerator dies, each with its own L2
constexpr int MK = 16;       // chunk of the inner dimension
constexpr int LDK = MK + 1;  // padded LDS row
constexpr int MT = 64;       // tile edge of the reference shape (sets the row split of gemm_hn)

// Work-groups are handed to the dies round-robin in the order of their
// linear index.  With grouping on, linear index L is mapped to logical
// index L' so that die d runs the contiguous logical range
// [start(d), start(d+1)), start(d) = d floor(N/8) + min(d, N mod 8): logical
// neighbours (the output tiles that read the same block of the large
// operand) then run on one die and share its L2.
__device__ __forceinline__ int64_t xcd_order(int64_t L, int64_t N, int group) {
  if (!group) return L;
  const int64_t d = L % kXcds, j = L / kXcds, q = N / kXcds, r = N % kXcds;
  return d * q + (d < r ? d : r) + j;
}

__device__ __forceinline__ int64_t linear_block() {
  return blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
}

}  // namespace

// Partial tiles of gemm_hn, independent of the tile shape: per (batch, split)
// the 16 x 16 blocks of the a x b result, block (bi, bj) at (bj nbi + bi) 256,
// inside a block lane l's slot s at 4 l + s (the MFMA result layout).
template <typename T, int WR, int WC, int BU, int BV>
__global__ void __launch_bounds__(256) k_gemm_hn_mfma(int64_t n, int a, int b, const cplx<T>* __restrict__ A,
                                                      int64_t lda, const cplx<T>* __restrict__ B, int64_t ldb,
                                                      int64_t rps, cplx<T>* __restrict__ part, int64_t sA,
                                                      int64_t sB, int group, Ragged rg) {
  constexpr int TR = WR * BU * 16, TC = WC * BV * 16, NLA = TR / 16, NLB = TC / 16;
  __shared__ T lds[2 * (TR + TC) * LDK];
  T* Ar = lds;
  T* Ai = Ar + TR * LDK;
  T* Br = Ai + TR * LDK;
  T* Bi = Br + TC * LDK;
  using M = Mfma<T>;
  using acc_t = typename M::acc;
  const int tiles_a = (a + TR - 1) / TR, tiles_b = (b + TC - 1) / TC;
  const int tiles = tiles_a * tiles_b;
  // logical order: the tiles of one row block (all tb) consecutive
  const int64_t lg = xcd_order(linear_block(), (int64_t)gridDim.x * gridDim.y * gridDim.z, group);
  const int tb = (int)(lg % tiles_b), ta = (int)((lg / tiles_b) % tiles_a);
  const int split = (int)((lg / tiles) % gridDim.y), batch = (int)(lg / ((int64_t)tiles * gridDim.y));
  if (rg.rows) {
    // ragged batch: entry `batch` is k-point k (kmap[batch], or batch), whose
    // n_k rows start at row off_k of the stacked A (A_k at A + a off_k,
    // leading dimension n_k); B_k is stacked the same way, or padded (at
    // B + k sB with leading dimension ldb)
    const int k = rg.kmap ? rg.kmap[batch] : batch;
    n = rg.rows[2 * k];
    const int64_t off = rg.rows[2 * k + 1];
    A += a * off;
    lda = n;
    if (rg.stacked) {
      B += b * off;
      ldb = n;
    } else {
      B += k * sB;
    }
  } else {
    A += batch * sA;
    B += batch * sB;
  }
  const int64_t r0 = split * rps, r1 = min(n, r0 + rps);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w % WR) * BU * 16, wj = (w / WR) * BV * 16;
  acc_t cre[BU][BV], cim[BU][BV];
#pragma unroll
  for (int u = 0; u < BU; ++u)
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      cre[u][v] = acc_t{0, 0, 0, 0};
      cim[u][v] = acc_t{0, 0, 0, 0};
    }
  // loader: thread t takes inner index t % 16 of columns t / 16 + 16 i
  const int lk = t & 15, lc = t >> 4;
  const int ia0 = ta * TR + lc, jb0 = tb * TC + lc;
  const cplx<T>* Ac = A + (int64_t)ia0 * lda + lk;
  const cplx<T>* Bc = B + (int64_t)jb0 * ldb + lk;
  // in single precision the next chunk is loaded into registers while the
  // current one is multiplied; in double precision it is loaded and stored
  // directly (the extra registers would cost occupancy)
  constexpr bool kPre = sizeof(T) == 4;
  cplx<T> pa[NLA], pb[NLB];
  auto fetch = [&](int64_t r) __attribute__((always_inline)) {
    const bool rok = r + lk < r1;
#pragma unroll
    for (int i = 0; i < NLA; ++i)
      pa[i] = (rok && ia0 + 16 * i < a) ? Ac[r + (int64_t)16 * i * lda] : mk<T>(0, 0);
#pragma unroll
    for (int i = 0; i < NLB; ++i)
      pb[i] = (rok && jb0 + 16 * i < b) ? Bc[r + (int64_t)16 * i * ldb] : mk<T>(0, 0);
  };
  if constexpr (kPre) {
    if (r0 < r1) fetch(r0);
  }
  for (int64_t r = r0; r < r1; r += MK) {
    if constexpr (!kPre) fetch(r);
#pragma unroll
    for (int i = 0; i < NLA; ++i) {
      Ar[(lc + 16 * i) * LDK + lk] = pa[i].x;
      Ai[(lc + 16 * i) * LDK + lk] = pa[i].y;
    }
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      Br[(lc + 16 * i) * LDK + lk] = pb[i].x;
      Bi[(lc + 16 * i) * LDK + lk] = pb[i].y;
    }
    __syncthreads();
    if constexpr (kPre) {
      if (r + MK < r1) fetch(r + MK);
    }
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      T ar[BU], ai[BU], br[BV], bi[BV];
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        ar[u] = Ar[(wi + 16 * u + cc) * LDK + kr];
        ai[u] = Ai[(wi + 16 * u + cc) * LDK + kr];
      }
#pragma unroll
      for (int v = 0; v < BV; ++v) {
        br[v] = Br[(wj + 16 * v + cc) * LDK + kr];
        bi[v] = Bi[(wj + 16 * v + cc) * LDK + kr];
      }
      // every accumulator takes one product before any takes its second, so
      // consecutive MFMAs are independent
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int v = 0; v < BV; ++v) {
          cre[u][v] = M::mma(ar[u], br[v], cre[u][v]);
          cim[u][v] = M::mma(ar[u], bi[v], cim[u][v]);
        }
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int v = 0; v < BV; ++v) {
          cre[u][v] = M::mma(ai[u], bi[v], cre[u][v]);
          cim[u][v] = M::mma(-ai[u], br[v], cim[u][v]);
        }
    }
    __syncthreads();
  }
  const int nbi = (a + 15) / 16, nbj = (b + 15) / 16;
  cplx<T>* P = part + ((int64_t)batch * gridDim.y + split) * ((int64_t)nbi * nbj * 256);
#pragma unroll
  for (int u = 0; u < BU; ++u)
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int bi = (ta * TR + wi) / 16 + u, bj = (tb * TC + wj) / 16 + v;
      if (bi < nbi && bj < nbj) {
        cplx<T>* Q = P + ((int64_t)bj * nbi + bi) * 256 + lane * 4;
#pragma unroll
        for (int s = 0; s < 4; ++s) Q[s] = mk<T>(cre[u][v][s], cim[u][v][s]);
      }
    }
}

// C = alpha sum_splits(partials) + beta C.  A work-group takes 16 consecutive
// partial positions; its 16 groups of 16 threads sum every 16th split each
// (independent loads in flight), and the 16 group sums are added in a fixed
// order, so the result does not depend on timing.
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_hn_mfma_reduce(int a, int b, int nsplit, const cplx<T>* __restrict__ part,
                                                             cplx<T>* C, int64_t ldc, double alpha, double beta,
                                                             int64_t sC) {
  using M = Mfma<T>;
  __shared__ double sx[16][17], sy[16][17];
  const int nbi = (a + 15) / 16, nbj = (b + 15) / 16;
  const int64_t per_split = (int64_t)nbi * nbj * 256;
  const int batch = blockIdx.y;
  C += batch * sC;
  const cplx<T>* P = part + (int64_t)batch * nsplit * per_split;
  const int j = threadIdx.x & 15, g = threadIdx.x >> 4;
  for (int64_t f0 = (int64_t)blockIdx.x * 16; f0 < per_split; f0 += (int64_t)gridDim.x * 16) {
    const int64_t f = f0 + j;
    double ax = 0, ay = 0;
    if (f < per_split) {
      for (int sp = g; sp < nsplit; sp += 16) {
        const cplx<T> v = P[sp * per_split + f];
        ax += (double)v.x;
        ay += (double)v.y;
      }
    }
    sx[g][j] = ax;
    sy[g][j] = ay;
    __syncthreads();
    if (g == 0 && f < per_split) {
      double tx = 0, ty = 0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        tx += sx[q][j];
        ty += sy[q][j];
      }
      const int s = (int)(f & 3), lane = (int)((f >> 2) & 63);
      const int64_t blk = f >> 8;
      const int bi = (int)(blk % nbi), bj = (int)(blk / nbi);
      const int i = bi * 16 + M::row(lane, s);
      const int jj = bj * 16 + (lane & 15);
      if (i < a && jj < b) {
        cplx<T>* c = C + i + (int64_t)jj * ldc;
        cplx<T> o;
        if (beta == 0.0) o = mk<T>((T)(alpha * tx), (T)(alpha * ty));
        else o = mk<T>((T)(alpha * tx + beta * (double)c->x), (T)(alpha * ty + beta * (double)c->y));
        *c = o;
      }
    }
    __syncthreads();
  }
}

template <typename T, int WR, int WC, int BU, int BV>
__global__ void __launch_bounds__(256) k_gemm_nn_mfma(int64_t n, int a, int b, const cplx<T>* __restrict__ A,
                                                      int64_t lda, const cplx<T>* __restrict__ Mm, int64_t ldm,
                                                      int opM, cplx<T>* __restrict__ C, int64_t ldc, double are,
                                                      double aim, double beta, int64_t sA, int64_t sM, int64_t sC,
                                                      int group, Ragged rg) {
  constexpr int TR = WR * BU * 16, TC = WC * BV * 16, NLA = TR / 16, NLB = TC / 16;
  // input planes; reused as the TR x 16 output staging tile (complex, row fastest)
  constexpr int kPlanes = 2 * (TR + TC) * LDK, kStage = 2 * 16 * (TR + 1);
  __shared__ T lds[kPlanes > kStage ? kPlanes : kStage];
  T* Ar = lds;
  T* Ai = Ar + TR * LDK;
  T* Mr = Ai + TR * LDK;
  T* Mi = Mr + TC * LDK;
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc;
  // logical order: the column tiles of one row block of A consecutive
  const int64_t lg = xcd_order(linear_block(), (int64_t)gridDim.x * gridDim.y * gridDim.z, group);
  const int tcol = (int)(lg % gridDim.y);
  const int64_t trow = (lg / gridDim.y) % gridDim.x;
  const int batch = (int)(lg / ((int64_t)gridDim.x * gridDim.y));
  Mm += batch * sM;
  if (rg.rows) {
    // ragged batch (as in k_gemm_hn_mfma): A_k stacked; C_k stacked (at
    // C + b off_k, leading dimension n_k) or padded (at C + k sC, ldc)
    const int k = rg.kmap ? rg.kmap[batch] : batch;
    n = rg.rows[2 * k];
    const int64_t off = rg.rows[2 * k + 1];
    A += a * off;
    lda = n;
    if (rg.stacked) {
      C += b * off;
      ldc = n;
    } else {
      C += k * sC;
    }
  } else {
    A += batch * sA;
    C += batch * sC;
  }
  const int64_t row0 = trow * TR;
  if (row0 >= n) return;  // a row tile beyond this entry's rows (uniform over the work-group)
  const int col0 = tcol * TC;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w % WR) * BU * 16, wj = (w / WR) * BV * 16;
  acc_t cre[BU][BV], cim[BU][BV];
#pragma unroll
  for (int u = 0; u < BU; ++u)
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      cre[u][v] = acc_t{0, 0, 0, 0};
      cim[u][v] = acc_t{0, 0, 0, 0};
    }
  // A loader: element e = t + 256 i of the TR x 16 chunk is row e % TR, inner
  // index e / TR (rows fastest, coalesced); M loader: element e of the
  // 16 x TC chunk is inner index e % 16, column e / 16 (M) or column e % TC,
  // inner index e / TC (M^H, whose columns are rows in memory)
  constexpr bool kPre = sizeof(T) == 4;
  cplx<T> pa[NLA], pm[NLB];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NLA; ++i) {
      const int e = t + 256 * i, k = k0 + e / TR;
      const int64_t row = row0 + e % TR;
      pa[i] = (row < n && k < a) ? A[row + (int64_t)k * lda] : mk<T>(0, 0);
    }
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      const int e = t + 256 * i;
      cplx<T> mv = mk<T>(0, 0);
      if (opM == 0) {
        const int k = k0 + (e & 15), j = col0 + (e >> 4);
        if (j < b && k < a) mv = Mm[k + (int64_t)j * ldm];
      } else {
        const int k = k0 + e / TC, j = col0 + e % TC;
        if (j < b && k < a) {
          const cplx<T> x = Mm[j + (int64_t)k * ldm];
          mv = mk<T>(x.x, -x.y);
        }
      }
      pm[i] = mv;
    }
  };
  if (kPre && a > 0) fetch(0);
  for (int k0 = 0; k0 < a; k0 += MK) {
    if (!kPre) fetch(k0);
#pragma unroll
    for (int i = 0; i < NLA; ++i) {
      const int e = t + 256 * i;
      Ar[(e % TR) * LDK + e / TR] = pa[i].x;
      Ai[(e % TR) * LDK + e / TR] = pa[i].y;
    }
#pragma unroll
    for (int i = 0; i < NLB; ++i) {
      const int e = t + 256 * i;
      const int jj = opM == 0 ? (e >> 4) : e % TC, kk = opM == 0 ? (e & 15) : e / TC;
      Mr[jj * LDK + kk] = pm[i].x;
      Mi[jj * LDK + kk] = pm[i].y;
    }
    __syncthreads();
    if (kPre && k0 + MK < a) fetch(k0 + MK);
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      T ar[BU], ai[BU], mr[BV], mi[BV];
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        ar[u] = Ar[(wi + 16 * u + cc) * LDK + kr];
        ai[u] = Ai[(wi + 16 * u + cc) * LDK + kr];
      }
#pragma unroll
      for (int v = 0; v < BV; ++v) {
        mr[v] = Mr[(wj + 16 * v + cc) * LDK + kr];
        mi[v] = Mi[(wj + 16 * v + cc) * LDK + kr];
      }
      // one product per accumulator before the second (independent consecutive MFMAs)
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int v = 0; v < BV; ++v) {
          cre[u][v] = Mf::mma(ar[u], mr[v], cre[u][v]);
          cim[u][v] = Mf::mma(ar[u], mi[v], cim[u][v]);
        }
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int v = 0; v < BV; ++v) {
          cre[u][v] = Mf::mma(-ai[u], mi[v], cre[u][v]);
          cim[u][v] = Mf::mma(ai[u], mr[v], cim[u][v]);
        }
    }
    __syncthreads();
  }
  // epilogue: 16 columns at a time through LDS, St[col][row] (row fastest,
  // stride TR + 1); the waves of one wave column write, all threads store
  cplx<T>* St = reinterpret_cast<cplx<T>*>(lds);
  constexpr int SLD = TR + 1;
#pragma unroll
  for (int wc = 0; wc < WC; ++wc)
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      if (w / WR == wc) {
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
          for (int s = 0; s < 4; ++s)
            St[(lane & 15) * SLD + wi + 16 * u + Mf::row(lane, s)] = mk<T>(cre[u][v][s], cim[u][v][s]);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < TR / 16; ++i) {
        const int e = t + 256 * i, rr = e % TR, cc = e / TR;
        const int64_t gi = row0 + rr;
        const int j = col0 + wc * BV * 16 + v * 16 + cc;
        if (gi < n && j < b) {
          const cplx<T> x = St[cc * SLD + rr];
          cplx<T>* c = C + gi + (int64_t)j * ldc;
          double ox = are * (double)x.x - aim * (double)x.y, oy = are * (double)x.y + aim * (double)x.x;
          if (beta != 0.0) {
            ox += beta * (double)c->x;
            oy += beta * (double)c->y;
          }
          *c = mk<T>((T)ox, (T)oy);
        }
      }
      __syncthreads();
    }
}

namespace {

// ---------------------------------------------------------------- shapes
struct Shape {
  int wr, wc, bu, bv;
  int tr() const { return wr * bu * 16; }
  int tc() const { return wc * bv * 16; }
};

// candidate 0 is the default (64 x 64)
template <typename T>
struct Shapes;
// (the last two, 64 x 32 and 64 x 16, are the narrow shapes for outputs of
// at most 32 and 16 columns)
#define EAHP_GEMM_SHAPES_F32(X) \
  X(2, 2, 2, 2) X(2, 2, 4, 2) X(2, 2, 2, 4) X(2, 2, 4, 4) X(4, 1, 2, 9) X(4, 1, 4, 4) X(4, 1, 1, 2) X(4, 1, 1, 1)
#define EAHP_GEMM_SHAPES_F64(X) X(2, 2, 2, 2) X(2, 2, 4, 2) X(2, 2, 2, 4) X(4, 1, 1, 2) X(4, 1, 1, 1)

using HnFn = void (*)(hipStream_t, dim3, int64_t, int, int, const void*, int64_t, const void*, int64_t, int64_t, void*,
                      int64_t, int64_t, int, Ragged);
using NnFn = void (*)(hipStream_t, dim3, int64_t, int, int, const void*, int64_t, const void*, int64_t, int, void*,
                      int64_t, double, double, double, int64_t, int64_t, int64_t, int, Ragged);

template <typename T, int WR, int WC, int BU, int BV>
void launch_hn(hipStream_t st, dim3 g, int64_t n, int a, int b, const void* A, int64_t lda, const void* B, int64_t ldb,
               int64_t rps, void* part, int64_t sA, int64_t sB, int group, Ragged rg) {
  hipLaunchKernelGGL((k_gemm_hn_mfma<T, WR, WC, BU, BV>), g, dim3(256), 0, st, n, a, b,
                     static_cast<const cplx<T>*>(A), lda, static_cast<const cplx<T>*>(B), ldb, rps,
                     static_cast<cplx<T>*>(part), sA, sB, group, rg);
}
template <typename T, int WR, int WC, int BU, int BV>
void launch_nn(hipStream_t st, dim3 g, int64_t n, int a, int b, const void* A, int64_t lda, const void* M, int64_t ldm,
               int opM, void* C, int64_t ldc, double are, double aim, double beta, int64_t sA, int64_t sM, int64_t sC,
               int group, Ragged rg) {
  hipLaunchKernelGGL((k_gemm_nn_mfma<T, WR, WC, BU, BV>), g, dim3(256), 0, st, n, a, b,
                     static_cast<const cplx<T>*>(A), lda, static_cast<const cplx<T>*>(M), ldm, opM,
                     static_cast<cplx<T>*>(C), ldc, are, aim, beta, sA, sM, sC, group, rg);
}

template <typename T>
struct ShapeTable {
  std::vector<Shape> shape;
  std::vector<HnFn> hn;
  std::vector<NnFn> nn;
};

#define EAHP_GEMM_ADD(WR, WC, BU, BV)                        \
  t.shape.push_back(Shape{WR, WC, BU, BV});                  \
  t.hn.push_back(&launch_hn<T, WR, WC, BU, BV>);             \
  t.nn.push_back(&launch_nn<T, WR, WC, BU, BV>);

template <typename T>
const ShapeTable<T>& shapes() {
  static const ShapeTable<T> tab = [] {
    ShapeTable<T> t;
    if constexpr (sizeof(T) == 4) {
      EAHP_GEMM_SHAPES_F32(EAHP_GEMM_ADD)
    } else {
      EAHP_GEMM_SHAPES_F64(EAHP_GEMM_ADD)
    }
    return t;
  }();
  return tab;
}
#undef EAHP_GEMM_ADD

// shape class of a product for the autotuner: each size rounded up to the
// next of 64, 96, 128, 192, 256, 384, ... (half-octave steps)
int64_t size_class(int64_t x) {
  int64_t c = 64;
  while (c < x) c = (c & (c - 1)) == 0 ? c + c / 2 : c / 3 * 4;
  return c;
}
// products below this many flops take the default shape without tuning
constexpr double kTuneMinFlops = 2e10;
std::string tune_key(const char* op, int fp32, int64_t n, int a, int b, int batch) {
  return std::string("gemm_") + op + (fp32 ? " f32" : " f64") + " n" + std::to_string(size_class(n)) + " a" +
         std::to_string(size_class(a)) + " b" + std::to_string(size_class(b)) + (batch > 1 ? " batched" : "");
}

}  // namespace

// Resident work-groups of the reference shape on the whole chip (CUs times
// work-groups per CU), queried once per precision.
template <typename T>
static int64_t hn_slots() {
  static const int64_t slots = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCK(hipGetDevice(&dev));
    HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, reinterpret_cast<const void*>(&k_gemm_hn_mfma<T, 2, 2, 2, 2>), 256, 0));
    return (int64_t)std::max(1, ncu) * std::max(1, per);
  }();
  return slots;
}

// Split of the row dimension (set with the reference 64 x 64 tiles, the same
// for every tile shape, so that all shapes give the same bits).  Tall
// products (n >= kTallRows): from the smallest count that keeps a split
// within max_rows, the count whose work-groups fill their last round of
// resident work-groups best (a count that leaves the last round mostly empty
// costs nearly a whole round).  Shorter ones, where a
// split holds few rows and the fixed cost of a work-group weighs more: about
// four work-groups per CU.  Always at least 4 chunks of rows per split, the
// partial tiles (written and read once more) under half the input bytes, and
// at most max_part complex partial values in all.
constexpr int64_t kTallRows = 16384;
// rows summed in the precision of the product per split of a tall product:
// FP32 sums are kept to 4096 rows (the splits are added in FP64)
template <typename T>
constexpr int64_t hn_max_rows() {
  return sizeof(T) == 4 ? 4096 : INT64_MAX / 2;
}
static void hn_split(int64_t n, int a, int b, int batch, int64_t max_part, int64_t slots, int64_t max_rows,
                     int64_t& nsplit, int64_t& rps, int64_t& per_split) {
  const int tiles = ((a + MT - 1) / MT) * ((b + MT - 1) / MT);
  const int64_t in_elems = n * (int64_t)(a + b);
  per_split = (int64_t)((a + 15) / 16) * ((b + 15) / 16) * 256;
  int64_t nmax = (n + 4 * MK - 1) / (4 * MK);
  nmax = std::min<int64_t>(nmax, std::max<int64_t>(1, in_elems / (2LL * tiles * MT * MT)));
  nmax = std::min<int64_t>(nmax, max_part / std::max<int64_t>(1, per_split * batch));
  nmax = std::max<int64_t>(1, nmax);
  const int64_t w0 = (int64_t)tiles * batch;
  auto fill = [&](int64_t ns) {
    const int64_t wg = w0 * ns;
    return (double)wg / (double)(((wg + slots - 1) / slots) * slots);
  };
  if (n >= kTallRows) {
    // single precision sums each split's rows in FP32: at most max_rows per split
    const int64_t nmin = std::min<int64_t>(nmax, (n + max_rows - 1) / max_rows);
    nsplit = nmin;
    double best = fill(nmin);
    const int64_t upto = std::min<int64_t>(nmax, std::max<int64_t>(nmin, 4 * slots / std::max<int64_t>(1, w0) + 1));
    for (int64_t ns = nmin + 1; ns <= upto; ++ns) {
      const double f = fill(ns);
      if (f > best + 0.02) {
        best = f;
        nsplit = ns;
      }
    }
  } else {
    nsplit = std::min<int64_t>(nmax, (1024 + w0 - 1) / w0);
  }
  rps = (n + nsplit - 1) / nsplit;
  rps = ((rps + MK - 1) / MK) * MK;
  nsplit = std::max<int64_t>(1, (n + rps - 1) / rps);
  if (n <= 0) {
    nsplit = 1;
    rps = 0;
  }
}

// die-grouped tile order of the products (on by default)
static std::atomic<int> g_xcd_group{1};
void gemm_set_xcd_group(int on) { g_xcd_group.store(on ? 1 : 0); }

size_t gemm_hn_min_part(int a, int b, int batch) {
  return (size_t)((a + 15) / 16) * ((b + 15) / 16) * 256 * batch;
}

int gemm_shape_count(int fp32) { return fp32 ? (int)shapes<float>().shape.size() : (int)shapes<double>().shape.size(); }

template <typename T>
static void hn_launch(hipStream_t st, int c, int64_t n, int a, int b, const cplx<T>* A, int64_t lda,
                      const cplx<T>* B, int64_t ldb, int64_t rps, int64_t nsplit, cplx<T>* part, int batch,
                      int64_t sA, int64_t sB, Ragged rg = Ragged{}) {
  const auto& tab = shapes<T>();
  const Shape& sh = tab.shape[c];
  const int tiles = ((a + sh.tr() - 1) / sh.tr()) * ((b + sh.tc() - 1) / sh.tc());
  tab.hn[c](st, dim3(tiles, (unsigned)nsplit, batch), n, a, b, A, lda, B, ldb, rps, part, sA, sB, g_xcd_group.load(),
            rg);
  HIPCK(hipGetLastError());
}

template <typename T>
static void hn_reduce(hipStream_t st, int a, int b, int64_t nsplit, int64_t per_split, const cplx<T>* part,
                      cplx<T>* C, int64_t ldc, double alpha, double beta, int batch, int64_t sC) {
  const int nb = (int)std::min<int64_t>(4096, (per_split + 15) / 16);
  hipLaunchKernelGGL((k_gemm_hn_mfma_reduce<T>), dim3(nb, batch), dim3(256), 0, st, a, b, (int)nsplit, part, C, ldc,
                     alpha, beta, sC);
  HIPCK(hipGetLastError());
}

// The tile shape of a product: the forced one, else the autotuner's for the
// shape class (tuned here on first use when tuning is on and `tune` allows:
// the candidates run on scratch outputs only), else the default.
template <typename T>
static int pick_shape(hipStream_t st, const char* op, int64_t n, int a, int b, int batch, bool tune,
                      const std::function<void(int)>& run) {
  const int nc = (int)shapes<T>().shape.size();
  const int f = autotune_forced();
  if (f >= 0) return std::min(f, nc - 1);
  // a narrow shape for outputs of at most 16 or 32 columns (a 64-column tile
  // would spend three quarters or half of its products on zeros); small
  // products otherwise take the 64 x 64 reference untimed
  if (b <= 16) return nc - 1;
  if (b <= 32) return nc - 2;
  if (8.0 * (double)n * a * b * batch < kTuneMinFlops) return 0;
  const std::string key = tune_key(op, sizeof(T) == 4, n, a, b, batch);
  return std::min(tune ? autotune(st, key, nc, run) : autotune_kept(key), nc - 1);
}

template <typename T>
void gemm_hn_mfma_ws(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                     int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, cplx<T>* part, size_t part_elems,
                     int batch, int64_t sA, int64_t sB, int64_t sC) {
  int64_t nsplit, rps, per_split;
  hn_split(n, a, b, batch, (int64_t)part_elems, hn_slots<T>(), hn_max_rows<T>(), nsplit, rps, per_split);
  if ((size_t)(nsplit * per_split * batch) > part_elems) fail(EAHP_EINVAL, "Gram product: partial buffer too small");
  // no tuning here (no allocation, no synchronisation): the kept choice
  const int c = pick_shape<T>(st, "hn", n, a, b, batch, false, nullptr);
  hn_launch<T>(st, c, n, a, b, A, lda, B, ldb, rps, nsplit, part, batch, sA, sB);
  hn_reduce<T>(st, a, b, nsplit, per_split, part, C, ldc, alpha, beta, batch, sC);
}

template <typename T>
void gemm_hn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                  int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch,
                  int64_t sA, int64_t sB, int64_t sC) {
  int64_t nsplit, rps, per_split;
  hn_split(n, a, b, batch, INT64_MAX, hn_slots<T>(), hn_max_rows<T>(), nsplit, rps, per_split);
  const size_t elems = (size_t)(nsplit * per_split * batch);
  part.ensure(sizeof(cplx<T>) * elems);
  cplx<T>* P = part.as<cplx<T>>();
  // candidates write only the partial tiles (scratch); the reduction is the same for all
  const int c = pick_shape<T>(st, "hn", n, a, b, batch, true, [&](int k) {
    hn_launch<T>(st, k, n, a, b, A, lda, B, ldb, rps, nsplit, P, batch, sA, sB);
  });
  hn_launch<T>(st, c, n, a, b, A, lda, B, ldb, rps, nsplit, P, batch, sA, sB);
  hn_reduce<T>(st, a, b, nsplit, per_split, P, C, ldc, alpha, beta, batch, sC);
}

template <typename T>
void gemm_nn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M,
                  int64_t ldm, int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta,
                  int batch, int64_t sA, int64_t sM, int64_t sC) {
  const auto& tab = shapes<T>();
  auto launch = [&](int k, cplx<T>* Cd, int64_t ldcd, int64_t sCd) {
    const Shape& sh = tab.shape[k];
    dim3 grid((unsigned)((n + sh.tr() - 1) / sh.tr()), (b + sh.tc() - 1) / sh.tc(), batch);
    tab.nn[k](st, grid, n, a, b, A, lda, M, ldm, opM, Cd, ldcd, alpha_re, alpha_im, beta, sA, sM, sC == 0 ? 0 : sCd,
              g_xcd_group.load(), Ragged{});
    HIPCK(hipGetLastError());
  };
  // candidates write a zeroed scratch output of the same size (same loads and stores)
  DevMem scratch;
  const int c = pick_shape<T>(st, "nn", n, a, b, batch, true, [&](int k) {
    if (!scratch.p) {
      scratch.alloc(sizeof(cplx<T>) * (size_t)n * b * batch);
      HIPCK(hipMemsetAsync(scratch.p, 0, sizeof(cplx<T>) * (size_t)n * b * batch, st));
    }
    launch(k, scratch.as<cplx<T>>(), n, n * (int64_t)b);
  });
  launch(c, C, ldc, sC);
}

// Ragged batches (see Ragged): the row split and the tile shape are those of
// one nmax-row product (nmax >= every n_k; the kept tile choice, no tuning);
// splits beyond an entry's rows add zeros.
template <typename T>
void gemm_hn_ragged_mfma(hipStream_t st, const Ragged& rg, int64_t nmax, int a, int b, const cplx<T>* A,
                         const cplx<T>* B, int64_t ldb, int64_t sB, cplx<T>* C, int64_t ldc, int64_t sC, double alpha,
                         double beta, DevMem& part, int batch) {
  int64_t nsplit, rps, per_split;
  hn_split(nmax, a, b, batch, INT64_MAX, hn_slots<T>(), hn_max_rows<T>(), nsplit, rps, per_split);
  part.ensure(sizeof(cplx<T>) * (size_t)(nsplit * per_split * batch));
  const int c = pick_shape<T>(st, "hn", nmax, a, b, batch, false, nullptr);
  hn_launch<T>(st, c, nmax, a, b, A, nmax, B, ldb, rps, nsplit, part.as<cplx<T>>(), batch, 0, sB, rg);
  hn_reduce<T>(st, a, b, nsplit, per_split, part.as<cplx<T>>(), C, ldc, alpha, beta, batch, sC);
}

template <typename T>
void gemm_nn_ragged_mfma(hipStream_t st, const Ragged& rg, int64_t nmax, int a, int b, const cplx<T>* A,
                         const cplx<T>* M, int64_t ldm, int64_t sM, int opM, cplx<T>* C, int64_t ldc, int64_t sC,
                         double alpha, double beta, int batch) {
  const auto& tab = shapes<T>();
  const int c = pick_shape<T>(st, "nn", nmax, a, b, batch, false, nullptr);
  const Shape& sh = tab.shape[c];
  dim3 grid((unsigned)((nmax + sh.tr() - 1) / sh.tr()), (b + sh.tc() - 1) / sh.tc(), batch);
  tab.nn[c](st, grid, nmax, a, b, A, nmax, M, ldm, opM, C, ldc, alpha, 0.0, beta, 0, sM, sC, g_xcd_group.load(), rg);
  HIPCK(hipGetLastError());
}

#define EAHP_RAGGED_INST(T)                                                                                         \
  template void gemm_hn_ragged_mfma<T>(hipStream_t, const Ragged&, int64_t, int, int, const cplx<T>*, const cplx<T>*, \
                                       int64_t, int64_t, cplx<T>*, int64_t, int64_t, double, double, DevMem&, int); \
  template void gemm_nn_ragged_mfma<T>(hipStream_t, const Ragged&, int64_t, int, int, const cplx<T>*, const cplx<T>*, \
                                       int64_t, int64_t, int, cplx<T>*, int64_t, int64_t, double, double, int);
EAHP_RAGGED_INST(double)
EAHP_RAGGED_INST(float)
#undef EAHP_RAGGED_INST
template void gemm_hn_mfma<double>(hipStream_t, int64_t, int, int, const z64*, int64_t, const z64*, int64_t, z64*,
                                   int64_t, double, double, DevMem&, int, int64_t, int64_t, int64_t);
template void gemm_hn_mfma_ws<double>(hipStream_t, int64_t, int, int, const z64*, int64_t, const z64*, int64_t, z64*,
                                      int64_t, double, double, z64*, size_t, int, int64_t, int64_t, int64_t);
template void gemm_hn_mfma<float>(hipStream_t, int64_t, int, int, const c32*, int64_t, const c32*, int64_t, c32*,
                                  int64_t, double, double, DevMem&, int, int64_t, int64_t, int64_t);
template void gemm_nn_mfma<double>(hipStream_t, int64_t, int, int, const z64*, int64_t, const z64*, int64_t, int,
                                   z64*, int64_t, double, double, double, int, int64_t, int64_t, int64_t);
template void gemm_nn_mfma<float>(hipStream_t, int64_t, int, int, const c32*, int64_t, const c32*, int64_t, int, c32*,
                                  int64_t, double, double, double, int, int64_t, int64_t, int64_t);

}  // namespace eahp
