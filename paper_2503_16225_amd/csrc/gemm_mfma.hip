// Complex block products on the matrix cores (v_mfma_*_16x16x4 in FP64 and
// FP32).  A complex product is four real ones on split real/imaginary planes:
//   A^H B : Re += ar br + ai bi,  Im += ar bi - ai br
//   A  M  : Re += ar mr - ai mi,  Im += ar mi + ai mr
// Operand layout of the 16x16x4 instructions (measured on gfx950): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; result slot s of lane l is
// element (4 s + l / 16, l % 16) in FP64 and (4 (l / 16) + s, l % 16) in FP32.
//
// gemm_hn (Gram matrices, Lambda, projector coefficients): the row dimension
// n is split over work-groups, each computes 64 x 64 output tiles over its
// rows and writes the raw fragments; a second kernel sums the splits in a
// fixed order (deterministic).
// gemm_nn (frame times small matrix): one 64 x 64 output tile per work-group,
// the inner dimension streamed through LDS 16 at a time, the tile staged
// through LDS for coalesced stores.
#include <atomic>

#include "devcommon.h"
#include "kernels.h"

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

constexpr int MT = 64;       // output tile edge
constexpr int kXcds = 8;     // MI355X: 8 accelerator dies, each with its own L2

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
constexpr int MK = 16;       // chunk of the inner dimension
constexpr int LDK = MK + 1;  // padded LDS row

}  // namespace

// Fragment layout of the partial tiles: for each (batch, split, tile, wave,
// u, v) a block of 64 lanes x 4 slots (complex).
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_hn_mfma(int64_t n, int a, int b, const cplx<T>* __restrict__ A,
                                                      int64_t lda, const cplx<T>* __restrict__ B, int64_t ldb,
                                                      int64_t rps, cplx<T>* __restrict__ part, int64_t sA,
                                                      int64_t sB, int group) {
  __shared__ T Ar[MT * LDK], Ai[MT * LDK], Br[MT * LDK], Bi[MT * LDK];
  using M = Mfma<T>;
  using acc_t = typename M::acc;
  const int tiles_a = (a + MT - 1) / MT;
  const int tiles = tiles_a * ((b + MT - 1) / MT);
  // logical order: the tiles of one column block of A (all tb) consecutive
  const int64_t nwg = (int64_t)gridDim.x * gridDim.y * gridDim.z;
  const int64_t lin = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t lg = xcd_order(lin, nwg, group);
  const int tiles_b = tiles / tiles_a;
  const int tb = (int)(lg % tiles_b), ta = (int)((lg / tiles_b) % tiles_a);
  const int split = (int)((lg / tiles) % gridDim.y), batch = (int)(lg / ((int64_t)tiles * gridDim.y));
  const int tile = ta + tiles_a * tb;
  A += batch * sA;
  B += batch * sB;
  const int64_t r0 = split * rps, r1 = min(n, r0 + rps);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      cre[u][v] = acc_t{0, 0, 0, 0};
      cim[u][v] = acc_t{0, 0, 0, 0};
    }
  const int lc = t >> 2, lr = (t & 3) * 4;
  const int ia = ta * MT + lc, jb = tb * MT + lc;
  const cplx<T>* Ac = A + (int64_t)min(ia, a - 1) * lda;
  const cplx<T>* Bc = B + (int64_t)min(jb, b - 1) * ldb;
  // in single precision the next chunk's rows are loaded into registers while
  // the current one is multiplied; in double precision the chunk is loaded
  // and stored directly (the extra registers would cost occupancy)
  constexpr bool kPre = sizeof(T) == 4;
  cplx<T> pa[4], pb[4];
  auto fetch = [&](int64_t r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = r + lr + q;
      pa[q] = mk<T>(0, 0);
      pb[q] = mk<T>(0, 0);
      if (row < r1) {
        if (ia < a) pa[q] = Ac[row];
        if (jb < b) pb[q] = Bc[row];
      }
    }
  };
  if constexpr (kPre) {
    if (r0 < r1) fetch(r0);
  }
  for (int64_t r = r0; r < r1; r += MK) {
    if constexpr (kPre) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Ar[lc * LDK + lr + q] = pa[q].x;
        Ai[lc * LDK + lr + q] = pa[q].y;
        Br[lc * LDK + lr + q] = pb[q].x;
        Bi[lc * LDK + lr + q] = pb[q].y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = r + lr + q;
        cplx<T> av = mk<T>(0, 0), bv = mk<T>(0, 0);
        if (row < r1) {
          if (ia < a) av = Ac[row];
          if (jb < b) bv = Bc[row];
        }
        Ar[lc * LDK + lr + q] = av.x;
        Ai[lc * LDK + lr + q] = av.y;
        Br[lc * LDK + lr + q] = bv.x;
        Bi[lc * LDK + lr + q] = bv.y;
      }
    }
    __syncthreads();
    if constexpr (kPre) {
      if (r + MK < r1) fetch(r + MK);
    }
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        ar[u] = Ar[(wi + 16 * u + cc) * LDK + kr];
        ai[u] = Ai[(wi + 16 * u + cc) * LDK + kr];
        br[u] = Br[(wj + 16 * u + cc) * LDK + kr];
        bi[u] = Bi[(wj + 16 * u + cc) * LDK + kr];
      }
      // the eight accumulators take one product each before any takes its
      // second, so consecutive MFMAs are independent
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          cre[u][v] = M::mma(ar[u], br[v], cre[u][v]);
          cim[u][v] = M::mma(ar[u], bi[v], cim[u][v]);
        }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          cre[u][v] = M::mma(ai[u], bi[v], cre[u][v]);
          cim[u][v] = M::mma(-ai[u], br[v], cim[u][v]);
        }
    }
    __syncthreads();
  }
  cplx<T>* P = part + ((((int64_t)batch * gridDim.y + split) * tiles + tile) * 4 + w) * 4 * 256;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int s = 0; s < 4; ++s) P[(u * 2 + v) * 256 + lane * 4 + s] = mk<T>(cre[u][v][s], cim[u][v][s]);
}

// C = alpha sum_splits(partials) + beta C.  A work-group takes 16 consecutive
// fragment positions; its 16 groups of 16 threads sum every 16th split each
// (independent loads in flight), and the 16 group sums are added in a fixed
// order, so the result does not depend on timing.
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_hn_mfma_reduce(int a, int b, int nsplit, const cplx<T>* __restrict__ part,
                                                             cplx<T>* C, int64_t ldc, double alpha, double beta,
                                                             int64_t sC) {
  using M = Mfma<T>;
  __shared__ double sx[16][17], sy[16][17];
  const int tiles_a = (a + MT - 1) / MT;
  const int tiles = tiles_a * ((b + MT - 1) / MT);
  const int64_t per_split = (int64_t)tiles * 4 * 4 * 256;
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
      const int s = (int)(f & 3), lane = (int)((f >> 2) & 63), uv = (int)((f >> 8) & 3), w = (int)((f >> 10) & 3);
      const int tile = (int)(f >> 12);
      const int ta = tile % tiles_a, tb = tile / tiles_a;
      const int i = ta * MT + (w & 1) * 32 + (uv >> 1) * 16 + M::row(lane, s);
      const int jj = tb * MT + (w >> 1) * 32 + (uv & 1) * 16 + (lane & 15);
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

template <typename T>
__global__ void __launch_bounds__(256) k_gemm_nn_mfma(int64_t n, int a, int b, const cplx<T>* __restrict__ A,
                                                      int64_t lda, const cplx<T>* __restrict__ Mm, int64_t ldm,
                                                      int opM, cplx<T>* __restrict__ C, int64_t ldc, double are,
                                                      double aim, double beta, int64_t sA, int64_t sM, int64_t sC,
                                                      int group) {
  // input planes; reused as the 64 x 32 output staging tile (complex, row fastest)
  __shared__ T lds[4 * MT * LDK];
  T* Ar = lds;
  T* Ai = Ar + MT * LDK;
  T* Mr = Ai + MT * LDK;
  T* Mi = Mr + MT * LDK;
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc;
  // logical order: the column tiles of one row block of A consecutive
  const int64_t nwg = (int64_t)gridDim.x * gridDim.y * gridDim.z;
  const int64_t lin = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t lg = xcd_order(lin, nwg, group);
  const int tcol = (int)(lg % gridDim.y);
  const int64_t trow = (lg / gridDim.y) % gridDim.x;
  const int batch = (int)(lg / ((int64_t)gridDim.x * gridDim.y));
  A += batch * sA;
  Mm += batch * sM;
  C += batch * sC;
  const int64_t row0 = trow * MT;
  const int col0 = tcol * MT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      cre[u][v] = acc_t{0, 0, 0, 0};
      cim[u][v] = acc_t{0, 0, 0, 0};
    }
  const int ak = t >> 4, arw = (t & 15) * 4;  // A loader: inner index ak, rows arw..arw+3
  const int mc = t >> 2, mq = (t & 3) * 4;    // M loader: column mc, inner indices mq..mq+3
  // the next chunk of A and M is loaded into registers while the current one
  // is multiplied (single precision only, as in k_gemm_hn_mfma)
  constexpr bool kPre = sizeof(T) == 4;
  cplx<T> pa[4], pm[4];
  auto fetch = [&](int k0) {
    const int k = k0 + ak;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = row0 + arw + q;
      pa[q] = (row < n && k < a) ? A[row + (int64_t)k * lda] : mk<T>(0, 0);
    }
    const int j = col0 + mc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kq = k0 + mq + q;
      cplx<T> mv = mk<T>(0, 0);
      if (j < b && kq < a) {
        if (opM == 0) mv = Mm[kq + (int64_t)j * ldm];
        else {
          const cplx<T> x = Mm[j + (int64_t)kq * ldm];
          mv = mk<T>(x.x, -x.y);
        }
      }
      pm[q] = mv;
    }
  };
  if (kPre && a > 0) fetch(0);
  for (int k0 = 0; k0 < a; k0 += MK) {
    if (!kPre) fetch(k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Ar[(arw + q) * LDK + ak] = pa[q].x;
      Ai[(arw + q) * LDK + ak] = pa[q].y;
      Mr[mc * LDK + mq + q] = pm[q].x;
      Mi[mc * LDK + mq + q] = pm[q].y;
    }
    __syncthreads();
    if (kPre && k0 + MK < a) fetch(k0 + MK);
#pragma unroll
    for (int kk = 0; kk < MK; kk += 4) {
      const int kr = kk + (lane >> 4), cc = lane & 15;
      T ar[2], ai[2], mr[2], mi[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        ar[u] = Ar[(wi + 16 * u + cc) * LDK + kr];
        ai[u] = Ai[(wi + 16 * u + cc) * LDK + kr];
        mr[u] = Mr[(wj + 16 * u + cc) * LDK + kr];
        mi[u] = Mi[(wj + 16 * u + cc) * LDK + kr];
      }
      // one product per accumulator before the second (independent consecutive MFMAs)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          cre[u][v] = Mf::mma(ar[u], mr[v], cre[u][v]);
          cim[u][v] = Mf::mma(ar[u], mi[v], cim[u][v]);
        }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          cre[u][v] = Mf::mma(-ai[u], mi[v], cre[u][v]);
          cim[u][v] = Mf::mma(ai[u], mr[v], cim[u][v]);
        }
    }
    __syncthreads();
  }
  // epilogue in two halves of 32 columns through LDS: St[col][row] (row fastest, stride 65)
  cplx<T>* St = reinterpret_cast<cplx<T>*>(lds);
  constexpr int SLD = MT + 1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if ((w >> 1) == h) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int rr = wi + 16 * u + Mf::row(lane, s);
            const int cc = 16 * v + (lane & 15);
            St[cc * SLD + rr] = mk<T>(cre[u][v][s], cim[u][v][s]);
          }
    }
    __syncthreads();
    {
      const int rr = t & 63;
      const int64_t i = row0 + rr;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int cc = (t >> 6) * 8 + q;
        const int j = col0 + h * 32 + cc;
        if (i < n && j < b) {
          const cplx<T> x = St[cc * SLD + rr];
          cplx<T>* c = C + i + (int64_t)j * ldc;
          double ox = are * (double)x.x - aim * (double)x.y, oy = are * (double)x.y + aim * (double)x.x;
          if (beta != 0.0) {
            ox += beta * (double)c->x;
            oy += beta * (double)c->y;
          }
          *c = mk<T>((T)ox, (T)oy);
        }
      }
    }
    __syncthreads();
  }
}

// Split of the row dimension: about four work-groups per CU (the loads of one
// overlap the products of the others), at least 4 chunks of rows each, the
// partial tiles (written and read once more) under half the input bytes, and
// at most max_part complex partial values in all.
static void hn_split(int64_t n, int a, int b, int batch, int64_t max_part, int64_t& nsplit, int64_t& rps,
                     int64_t& per_split) {
  const int tiles = ((a + MT - 1) / MT) * ((b + MT - 1) / MT);
  const int64_t in_elems = n * (int64_t)(a + b);
  per_split = (int64_t)tiles * 4 * 4 * 256;
  nsplit = (1024 + tiles * batch - 1) / (tiles * batch);
  nsplit = std::min<int64_t>(nsplit, (n + 4 * MK - 1) / (4 * MK));
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, in_elems / (2LL * tiles * MT * MT)));
  nsplit = std::min<int64_t>(nsplit, max_part / std::max<int64_t>(1, per_split * batch));
  nsplit = std::max<int64_t>(1, nsplit);
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
  const int tiles = ((a + MT - 1) / MT) * ((b + MT - 1) / MT);
  return (size_t)tiles * 4 * 4 * 256 * batch;
}

template <typename T>
void gemm_hn_mfma_ws(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                     int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, cplx<T>* part, size_t part_elems,
                     int batch, int64_t sA, int64_t sB, int64_t sC) {
  const int tiles = ((a + MT - 1) / MT) * ((b + MT - 1) / MT);
  int64_t nsplit, rps, per_split;
  hn_split(n, a, b, batch, (int64_t)part_elems, nsplit, rps, per_split);
  if ((size_t)(nsplit * per_split * batch) > part_elems) fail(EAHP_EINVAL, "Gram product: partial buffer too small");
  hipLaunchKernelGGL((k_gemm_hn_mfma<T>), dim3(tiles, (unsigned)nsplit, batch), dim3(256), 0, st, n, a, b, A, lda, B,
                     ldb, rps, part, sA, sB, g_xcd_group.load());
  HIPCK(hipGetLastError());
  const int nb = (int)std::min<int64_t>(4096, (per_split + 15) / 16);
  hipLaunchKernelGGL((k_gemm_hn_mfma_reduce<T>), dim3(nb, batch), dim3(256), 0, st, a, b, (int)nsplit, part, C, ldc,
                     alpha, beta, sC);
  HIPCK(hipGetLastError());
}

template <typename T>
void gemm_hn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                  int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch,
                  int64_t sA, int64_t sB, int64_t sC) {
  int64_t nsplit, rps, per_split;
  hn_split(n, a, b, batch, INT64_MAX, nsplit, rps, per_split);
  const size_t elems = (size_t)(nsplit * per_split * batch);
  part.ensure(sizeof(cplx<T>) * elems);
  gemm_hn_mfma_ws<T>(st, n, a, b, A, lda, B, ldb, C, ldc, alpha, beta, part.as<cplx<T>>(), elems, batch, sA, sB, sC);
}

template <typename T>
void gemm_nn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M,
                  int64_t ldm, int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta,
                  int batch, int64_t sA, int64_t sM, int64_t sC) {
  dim3 grid((unsigned)((n + MT - 1) / MT), (b + MT - 1) / MT, batch);
  hipLaunchKernelGGL((k_gemm_nn_mfma<T>), grid, dim3(256), 0, st, n, a, b, A, lda, M, ldm, opM, C, ldc, alpha_re,
                     alpha_im, beta, sA, sM, sC, g_xcd_group.load());
  HIPCK(hipGetLastError());
}

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
