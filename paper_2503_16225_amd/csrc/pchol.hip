// Diagonally pivoted Cholesky factorisation with rank cut-off and the inverse
// of the factor, for the rank-revealing orthonormalisation of the block FOM
// (CholQR on the Gram matrix of a block) and, unpivoted, for the qR
// retraction: G[piv, piv] = L L^H, pivots below
// tol times the first one end the factorisation (rank r), and the output is
// U = P L^-H (n x r; row piv[k] of U holds row k of L^-H), so that R U has
// orthonormal columns spanning the retained directions of R.
//
// One work-group of 1024 threads, n <= 128, the matrix in registers (thread t
// owns row t/8 and the 16 columns congruent to t mod 8).  Pivoting is logical
// (rows and columns are marked done instead of being exchanged); the pivot
// search is a shuffle reduction in every wave followed by a scan of the 16
// wave candidates in every thread, so a step takes two barriers.  The
// factor is written row-major to a scratch matrix; the inverse factor is a
// second launch, k_chol_uinv, with one wave per column of U (independent
// backward substitutions, no block barriers).
#include <mutex>

#include "devcommon.h"
#include "exchange.h"
#include "kernels.h"

namespace eahp {

namespace {
constexpr int kPcMax = 128;
__device__ __forceinline__ z64 cmulz(z64 a, z64 b) { return mk<double>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
}  // namespace

__global__ void __launch_bounds__(1024) k_pchol_reg(int n, const z64* __restrict__ G, int64_t ldg, double tol,
                                                    int* __restrict__ piv, int* __restrict__ rank_out,
                                                    z64* __restrict__ U, int64_t ldu, z64* __restrict__ Lg,
                                                    int pivot, int64_t sG) {
  // one matrix per work-group (blockIdx.x): G at stride sG, piv at n, rank at 1, Lg at n^2
  G += blockIdx.x * sG;
  piv += (int64_t)blockIdx.x * n;
  rank_out += blockIdx.x;
  Lg += (int64_t)blockIdx.x * n * n;
  __shared__ double cv[16];
  __shared__ int ci[16];
  __shared__ int done[kPcMax];
  __shared__ int pv[kPcMax];
  __shared__ z64 lcol[2][kPcMax];
  const int t = threadIdx.x;
  if (t < 2 * kPcMax) lcol[t >> 7][t & (kPcMax - 1)] = mk<double>(0.0, 0.0);
  const int rr = t >> 3, cg = t & 7, lane = t & 63, wv = t >> 6;
  d16 ar, ai;  // row rr, columns cg + 8 m (real and imaginary parts)
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = cg + 8 * m;
    z64 v = mk<double>(0.0, 0.0);
    if (rr < n && c < n) {
      const z64 x = G[rr + (int64_t)c * ldg], y = G[c + (int64_t)rr * ldg];
      v = mk<double>(0.5 * (x.x + y.x), rr == c ? 0.0 : 0.5 * (x.y - y.y));
    }
    ar[m] = v.x;
    ai[m] = v.y;
  }
  // the remaining diagonal of this thread's row (the same in the 8 lanes of the
  // row) and whether the row has been a pivot.  Rows and columns that are done
  // keep being updated: their entries are never read again.
  double dg = rr < n ? G[rr + (int64_t)rr * ldg].x : 0.0;
  bool isp = false;
  int r = n;
  double d0 = 0;
  for (int k = 0; k < n; ++k) {
    // pivot: largest remaining diagonal (ties: smallest index); arg-max in
    // every wave, then over the 16 wave candidates in every wave
    if (pivot) {
      const bool live = rr < n && !isp;
      double val = live ? dg : -1.0;
      int row = live ? rr : 1 << 20;
      wave_argmax(val, row);
      if (lane == 0) {
        cv[wv] = val;
        ci[wv] = row;
      }
    } else if (rr == k && cg == 0) {
      cv[0] = dg;  // pivots in order: row k
    }
    __syncthreads();
    double best;
    int b;
    if (pivot) {
      best = lane < 16 ? cv[lane] : -2.0;
      b = lane < 16 ? ci[lane] : 1 << 20;
      row16_argmax(best, b);
      best = readlane_f64(best, 0);
      b = __builtin_amdgcn_readlane(b, 0);
    } else {
      best = cv[0];
      b = k;
    }
    if (k == 0) d0 = best;
    if (!(best > tol * d0) || !(best > 0.0)) {
      r = k;
      break;
    }
    if (t == 0) pv[k] = b;
    const double lbb = sqrt(best);
    const double ilbb = 1.0 / lbb;
    // column b of the factor: l_i = a_ib / l_bb for the remaining rows, l_b = l_bb
    const int bm = __builtin_amdgcn_readfirstlane(b >> 3);
    const z64 ab = mk<double>(ar[bm], ai[bm]);
    z64 lv = rr == b ? mk<double>(lbb, 0.0) : (isp || rr >= n) ? mk<double>(0.0, 0.0) : cscale<double>(ab, ilbb);
    if (cg == (b & 7) && rr < n) {
      lcol[k & 1][rr] = lv;
      Lg[(int64_t)rr * n + k] = lv;  // row-major: l(rr, k)
    }
    // this row's l, from the lane of the row that holds column b
    const int src = (lane & ~7) | (b & 7);
    lv = mk<double>(__shfl(lv.x, src, 64), __shfl(lv.y, src, 64));
    if (rr == b) isp = true;
    __syncthreads();
    // a_rc -= l_r conj(l_c), reads of l in groups of four
#pragma unroll
    for (int mb = 0; mb < 16; mb += 4) {
      z64 lc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) lc[u] = lcol[k & 1][cg + 8 * (mb + u)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int m = mb + u;
        ar[m] = fma(-lv.x, lc[u].x, fma(-lv.y, lc[u].y, ar[m]));
        ai[m] = fma(-lv.y, lc[u].x, fma(lv.x, lc[u].y, ai[m]));
      }
    }
    dg -= lv.x * lv.x + lv.y * lv.y;
  }
  if (cg == 0 && rr < n) done[rr] = isp ? 1 : 0;
  __syncthreads();
  // remaining indices after the pivots, in increasing order
  if (t == 0) {
    // the pivots 0..r-1 are exactly the indices marked done
    int q = r;
    for (int i = 0; i < n; ++i)
      if (!done[i]) pv[q++] = i;
    *rank_out = r;
  }
  __syncthreads();
  for (int i = t; i < n; i += blockDim.x) piv[i] = pv[i];
}

// Column j < r of U = P L^-H: y = Lt^-H e_j with Lt[a][m] = l(piv[a], m) lower
// triangular in pivot order, by backward substitution over a = j .. 0 (lane
// l owns indices l and l + 64); U[piv[m]][j] = y_m for m <= j, 0 otherwise.
// One wave per column; row piv[a] of the factor is read contiguously and
// prefetched one step ahead.
__global__ void __launch_bounds__(64) k_chol_uinv(int n, const int* __restrict__ rank, const int* __restrict__ piv,
                                                  const z64* __restrict__ Lg, z64* __restrict__ U, int64_t ldu,
                                                  int64_t sU) {
  // matrix blockIdx.y: rank at 1, piv at n, Lg at n^2, U at sU
  rank += blockIdx.y;
  piv += (int64_t)blockIdx.y * n;
  Lg += (int64_t)blockIdx.y * n * n;
  U += blockIdx.y * sU;
  const int j = blockIdx.x, l = threadIdx.x;
  const int r = *rank;
  if (j >= r) return;
  __shared__ int pv[kPcMax];
  for (int i = l; i < n; i += 64) pv[i] = piv[i];
  __syncthreads();
  z64 rhs0 = mk<double>(l == j ? 1.0 : 0.0, 0.0), rhs1 = mk<double>(l + 64 == j ? 1.0 : 0.0, 0.0);
  z64 y0 = mk<double>(0.0, 0.0), y1 = mk<double>(0.0, 0.0);
  const z64 zero = mk<double>(0.0, 0.0);
  const z64* row = Lg + (int64_t)pv[j] * n;
  z64 c0 = l < n ? row[l] : zero, c1 = l + 64 < n ? row[l + 64] : zero;
  for (int a = j; a >= 0; --a) {
    const z64 a0 = c0, a1 = c1;
    if (a > 0) {  // next row, independent of this step's result
      const z64* nrow = Lg + (int64_t)pv[a - 1] * n;
      c0 = l < a - 1 + 1 ? nrow[l] : zero;
      c1 = l + 64 < a ? nrow[l + 64] : zero;
    }
    // y_a = rhs_a / Lt[a][a] in the lane that owns a, broadcast
    const bool lo = a < 64;
    const z64 ra = lo ? rhs0 : rhs1;
    const z64 da = lo ? a0 : a1;  // Lt[a][a] sits at the lane owning a
    const int own = a & 63;
    const double inv = 1.0 / __shfl(da.x, own, 64);
    const double yx = __shfl(ra.x, own, 64) * inv, yy = __shfl(ra.y, own, 64) * inv;
    if (l == own) {
      if (lo) y0 = mk<double>(yx, yy);
      else y1 = mk<double>(yx, yy);
    }
    // rhs_m -= conj(Lt[a][m]) y_a for m < a
    if (l < a) {
      rhs0.x -= a0.x * yx + a0.y * yy;
      rhs0.y -= a0.x * yy - a0.y * yx;
    }
    if (l + 64 < a) {
      rhs1.x -= a1.x * yx + a1.y * yy;
      rhs1.y -= a1.x * yy - a1.y * yx;
    }
  }
  if (l < n) U[pv[l] + (int64_t)j * ldu] = l <= j ? y0 : zero;
  if (l + 64 < n) U[pv[l + 64] + (int64_t)j * ldu] = l + 64 <= j ? y1 : zero;
}

bool pchol_inv_reg(hipStream_t st, int n, const z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* U,
                   int64_t ldu, DevMem& scr, bool pivot) {
  if (n < 1 || n > kPcMax) return false;
  scr.ensure(sizeof(z64) * (size_t)n * n);
  hipLaunchKernelGGL(k_pchol_reg, dim3(1), dim3(1024), 0, st, n, G, ldg, tol, piv, rank, U, ldu, scr.as<z64>(),
                     pivot ? 1 : 0, (int64_t)0);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_chol_uinv, dim3(n), dim3(64), 0, st, n, rank, piv, scr.as<z64>(), U, ldu, (int64_t)0);
  HIPCK(hipGetLastError());
  return true;
}

__global__ void k_zero_z(z64* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = mk<double>(0.0, 0.0);
}

// batch of pivoted factorisations (n <= 128, one work-group each): G at
// stride sG, piv (n each), rank (1 each), U (n x n each, stride sU; columns
// beyond the rank are zero)
void pchol_inv_batched(hipStream_t st, int n, const z64* G, int64_t ldg, int64_t sG, double tol, int* piv, int* rank,
                       z64* U, int64_t ldu, int64_t sU, int batch, DevMem& scr) {
  if (n < 1 || n > kPcMax) fail(EAHP_EINVAL, "batched pivoted Cholesky: n > 128");
  scr.ensure(sizeof(z64) * (size_t)n * n * batch);
  hipLaunchKernelGGL(k_zero_z, dim3((unsigned)std::min<int64_t>(1024, (sU * batch + 255) / 256)), dim3(256), 0, st, U,
                     sU * batch);
  hipLaunchKernelGGL(k_pchol_reg, dim3(batch), dim3(1024), 0, st, n, G, ldg, tol, piv, rank, U, ldu, scr.as<z64>(),
                     1, sG);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_chol_uinv, dim3(n, batch), dim3(64), 0, st, n, rank, piv, scr.as<z64>(), U, ldu, sU);
  HIPCK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// kPcMax < n <= kPcBig: the same factorisation (logical pivoting, the same
// pivot and rank rules, the factor written row-major to Lg) blocked by panels
// of kPb columns in one work-group, with the Schur complement in global
// memory (G, overwritten after Hermitisation).  Inside a panel a column needs
// only the panel's earlier columns, kept column-major in P (n x kPb) for
// coalesced reads; after the panel the live part of the trailing matrix takes
// the panel's rank-kPb update.
namespace {
constexpr int kPcBig = 2048;
constexpr int kPb = 16;
}  // namespace

__global__ void __launch_bounds__(512) k_pchol_big(int n, z64* G, int64_t ldg, double tol, int* __restrict__ piv,
                                                    int* __restrict__ rank_out, z64* __restrict__ Lg,
                                                    z64* __restrict__ P, int pivot) {
  __shared__ double dg[kPcBig];
  __shared__ int done[kPcBig];
  __shared__ int pvs[kPcBig];
  __shared__ z64 lp[kPb];
  __shared__ z64 ljs[8][kPb];  // panel row of each wave's column in the trailing update
  __shared__ double cv[16];
  __shared__ int ci[16];
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  for (int j = wv; j < n; j += (nt >> 6))
    for (int i = lane; i < j; i += 64) {
      const z64 a = G[i + (int64_t)j * ldg], b = G[j + (int64_t)i * ldg];
      const z64 h = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      G[i + (int64_t)j * ldg] = h;
      G[j + (int64_t)i * ldg] = mk<double>(h.x, -h.y);
    }
  for (int i = t; i < n; i += nt) {
    dg[i] = G[i + (int64_t)i * ldg].x;
    done[i] = 0;
  }
  __syncthreads();
  double d0 = 0.0;
  int r = n;
  for (int k0 = 0; k0 < n && r == n; k0 += kPb) {
    const int kend = min(n, k0 + kPb);
    int k = k0;
    for (; k < kend; ++k) {
      double best;
      int b;
      if (pivot) {
        double val = -1.0;
        int row = 1 << 20;
        for (int i = t; i < n; i += nt)
          if (!done[i] && dg[i] > val) {
            val = dg[i];
            row = i;
          }
        wave_argmax(val, row);
        if (lane == 0) {
          cv[wv] = val;
          ci[wv] = row;
        }
        __syncthreads();
        best = lane < (nt >> 6) ? cv[lane] : -2.0;
        b = lane < (nt >> 6) ? ci[lane] : 1 << 20;
        row16_argmax(best, b);
        best = readlane_f64(best, 0);
        b = __builtin_amdgcn_readlane(b, 0);
      } else {
        best = dg[k];
        b = k;
      }
      if (k == 0) d0 = best;
      if (!(best > tol * d0) || !(best > 0.0)) {
        r = k;
        break;
      }
      const double lbb = sqrt(best), il = 1.0 / lbb;
      const int np = k - k0;
      if (t < np) lp[t] = P[b + (int64_t)t * n];
      __syncthreads();
      for (int i = t; i < n; i += nt) {
        z64 l = mk<double>(0.0, 0.0);
        if (i == b) {
          l = mk<double>(lbb, 0.0);
        } else if (!done[i]) {
          z64 a = G[i + (int64_t)b * ldg];
          // the panel's earlier columns, loaded together (fixed trip count)
          z64 li[kPb];
#pragma unroll
          for (int c = 0; c < kPb; ++c) li[c] = c < np ? P[i + (int64_t)c * n] : mk<double>(0.0, 0.0);
#pragma unroll
          for (int c = 0; c < kPb; ++c) {
            if (c < np) {
              const z64 lb = lp[c];
              a.x -= li[c].x * lb.x + li[c].y * lb.y;
              a.y -= li[c].y * lb.x - li[c].x * lb.y;
            }
          }
          l = cscale<double>(a, il);
          dg[i] -= l.x * l.x + l.y * l.y;
        }
        P[i + (int64_t)np * n] = l;
        Lg[(int64_t)i * n + k] = l;
      }
      __syncthreads();
      if (t == 0) {
        done[b] = 1;
        pvs[k] = b;
      }
      __syncthreads();
    }
    const int np = k - k0;
    if (r == n && np > 0 && kend < n) {
      // live trailing entries: a wave per column j (its panel row in
      // registers, uniform over the wave), lanes over the rows i
      const int nw = nt >> 6;
      for (int j = wv; j < n; j += nw) {
        if (done[j]) continue;
        if (lane < kPb) ljs[wv][lane] = lane < np ? P[j + (int64_t)lane * n] : mk<double>(0.0, 0.0);
        __builtin_amdgcn_wave_barrier();
        z64* Gj = G + (int64_t)j * ldg;
        for (int i = lane; i < n; i += 64) {
          if (done[i]) continue;
          z64 a = Gj[i];
#pragma unroll
          for (int c = 0; c < kPb; ++c) {
            if (c < np) {
              const z64 li = P[i + (int64_t)c * n], lj = ljs[wv][c];
              a.x -= li.x * lj.x + li.y * lj.y;
              a.y -= li.y * lj.x - li.x * lj.y;
            }
          }
          Gj[i] = a;
        }
        __builtin_amdgcn_wave_barrier();
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    int q = r;
    for (int i = 0; i < n; ++i)
      if (!done[i]) pvs[q++] = i;
    *rank_out = r;
  }
  __syncthreads();
  for (int i = t; i < n; i += nt) piv[i] = pvs[i];
}

// Column j < r of U = P L^-H for n > kPcMax: the backward substitution of
// k_chol_uinv with the right-hand side in LDS, one work-group per column.
__global__ void __launch_bounds__(256) k_chol_uinv_big(int n, const int* __restrict__ rank,
                                                       const int* __restrict__ piv, const z64* __restrict__ Lg,
                                                       z64* __restrict__ U, int64_t ldu) {
  __shared__ z64 rhs[kPcBig];
  __shared__ int pv[kPcBig];
  __shared__ z64 ya;
  const int j = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
  const int r = *rank;
  if (j >= r) return;
  for (int i = t; i < n; i += nt) {
    pv[i] = piv[i];
    rhs[i] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int a = j; a >= 0; --a) {
    const z64* row = Lg + (int64_t)pv[a] * n;  // Lt[a][m] = row[m]
    if (t == 0) {
      const double inv = 1.0 / row[a].x;
      ya = mk<double>(rhs[a].x * inv, rhs[a].y * inv);
      rhs[a] = ya;
    }
    __syncthreads();
    const z64 y = ya;
    for (int m = t; m < a; m += nt) {
      const z64 c = row[m];
      rhs[m].x -= c.x * y.x + c.y * y.y;
      rhs[m].y -= c.x * y.y - c.y * y.x;
    }
    __syncthreads();
  }
  for (int i = t; i < n; i += nt) U[pv[i] + (int64_t)j * ldu] = i <= j ? rhs[i] : mk<double>(0.0, 0.0);
}

// kPcMax < n <= 64 NS on a cooperative grid of 8-wave work-groups: every wave
// holds two columns of the Schur complement in registers (row i in lane
// i % 64, slot i / 64); every work-group keeps the remaining diagonal and the
// pivot flags in LDS and chooses the same pivot (the same rules as above);
// the wave owning the pivot column publishes the factor column through
// exchange slots (row k of Xs for step k) that every work-group polls, then
// every wave updates its own columns.  No grid barrier; waits are bounded and
// a timeout is reported through *err.  The factor goes row-major to Lg.
template <int NS>
__global__ void __launch_bounds__(512) k_pchol_coop(int n, const z64* __restrict__ G, int64_t ldg, double tol,
                                                    int* __restrict__ piv, int* __restrict__ rank_out,
                                                    z64* __restrict__ Lg, z64* Xs, int* err, int pivot) {
  __shared__ double dg[64 * NS];
  __shared__ int done[64 * NS];
  __shared__ int pvs[64 * NS];
  __shared__ z64 lcol[64 * NS];
  __shared__ double cv[8];
  __shared__ int ci[8];
  __shared__ int sbad;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6), nwv = nt >> 6;
  const int nwt = gridDim.x * nwv, gw = blockIdx.x * nwv + wv;
  int col[2];
  z64 a[2][NS];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    col[j] = gw + j * nwt;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      z64 v = mk<double>(0.0, 0.0);
      if (col[j] < n && i < n) {
        const z64 x = G[i + (int64_t)col[j] * ldg], y = G[col[j] + (int64_t)i * ldg];
        v = mk<double>(0.5 * (x.x + y.x), i == col[j] ? 0.0 : 0.5 * (x.y - y.y));
      }
      a[j][s] = v;
    }
  }
  for (int i = t; i < n; i += nt) {
    dg[i] = G[i + (int64_t)i * ldg].x;
    done[i] = 0;
  }
  if (t == 0) sbad = 0;
  __syncthreads();
  double d0 = 0.0;
  int r = n;
  for (int k = 0; k < n; ++k) {
    double best;
    int b;
    if (pivot) {
      double val = -1.0;
      int row = 1 << 20;
      for (int i = t; i < n; i += nt)
        if (!done[i] && dg[i] > val) {
          val = dg[i];
          row = i;
        }
      wave_argmax(val, row);
      if (lane == 0) {
        cv[wv] = val;
        ci[wv] = row;
      }
      __syncthreads();
      best = cv[0];
      b = ci[0];
      for (int w = 1; w < nwv; ++w) argmax_merge(best, b, cv[w], ci[w]);
    } else {
      best = dg[k];
      b = k;
    }
    if (k == 0) d0 = best;
    if (!(best > tol * d0) || !(best > 0.0)) {
      r = k;
      break;
    }
    const double lbb = sqrt(best), il = 1.0 / lbb;
    // the owner of column b publishes l = S[:, b] / l_bb (0 on pivot rows, l_bb on b)
    const int jb = b / nwt, gb = b - jb * nwt;
    if (gw == gb) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = lane + 64 * s;
        if (i < n) {
          const z64 x = jb == 0 ? a[0][s] : a[1][s];
          const z64 l = i == b ? mk<double>(lbb, 0.0) : done[i] ? mk<double>(0.0, 0.0) : cscale<double>(x, il);
          xch::put_z(Xs + (int64_t)k * n + i, l);
          Lg[(int64_t)i * n + k] = l;
        }
      }
    }
    for (int i = t; i < n; i += nt) {
      bool ok = true;
      lcol[i] = xch::poll_z(Xs + (int64_t)k * n + i, ok);
      if (!ok) sbad = 1;
    }
    __syncthreads();
    if (sbad) {
      if (t == 0) *reinterpret_cast<volatile int*>(err) = 1;
      return;
    }
    for (int i = t; i < n; i += nt)
      if (!done[i]) {
        const z64 l = lcol[i];
        dg[i] -= l.x * l.x + l.y * l.y;
      }
    // own live columns: S[:, c] -= l conj(l_c)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = col[j];
      if (c < n && !done[c] && c != b) {
        const z64 lc = lcol[c];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int i = lane + 64 * s;
          const z64 l = i < n ? lcol[i] : mk<double>(0.0, 0.0);
          a[j][s].x -= l.x * lc.x + l.y * lc.y;
          a[j][s].y -= l.y * lc.x - l.x * lc.y;
        }
      }
    }
    __syncthreads();
    if (t == 0) {
      done[b] = 1;
      pvs[k] = b;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    if (t == 0) {
      int q = r;
      for (int i = 0; i < n; ++i)
        if (!done[i]) pvs[q++] = i;
      *rank_out = r;
    }
    __syncthreads();
    for (int i = t; i < n; i += nt) piv[i] = pvs[i];
  }
}

__global__ void k_fill_xch(unsigned long long* p, int64_t n, int* err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = xch::kEmpty;
  if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
}

template <int NS>
static void pchol_coop_launch(hipStream_t st, int n, const z64* G, int64_t ldg, double tol, int* piv, int* rank,
                              z64* Lg, z64* Xs, int* err, int pivot) {
  const int nwg = (n + 15) / 16;  // 8 waves x 2 columns per work-group
  const int64_t nw = (int64_t)2 * n * n;
  hipLaunchKernelGGL(k_fill_xch, dim3((unsigned)std::min<int64_t>(1024, (nw + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(Xs), nw, err);
  int nn = n;
  int64_t lg = ldg;
  void* args[] = {&nn, &G, &lg, &tol, &piv, &rank, &Lg, &Xs, &err, &pivot};
  HIPCK(hipLaunchCooperativeKernel((const void*)k_pchol_coop<NS>, dim3(nwg), dim3(512), args, 0, st));
}

bool pchol_inv_big(hipStream_t st, int n, z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* U, int64_t ldu,
                   DevMem& scr, bool pivot) {
  if (n <= kPcMax || n > kPcBig) return false;
  if (n <= 512) {
    // the factor (n^2), the exchange slots (n^2), the error flag
    scr.ensure(sizeof(z64) * 2 * (size_t)n * n + 64);
    z64* Lg = scr.as<z64>();
    z64* Xs = Lg + (size_t)n * n;
    int* err = reinterpret_cast<int*>(Xs + (size_t)n * n);
    {
      std::lock_guard<std::mutex> lk(coop_mutex());
      if (n <= 256) pchol_coop_launch<4>(st, n, G, ldg, tol, piv, rank, Lg, Xs, err, pivot ? 1 : 0);
      else pchol_coop_launch<8>(st, n, G, ldg, tol, piv, rank, Lg, Xs, err, pivot ? 1 : 0);
      int bad = 0;
      HIPCK(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCK(hipStreamSynchronize(st));
      if (bad) fail(EAHP_EDEVICE, "exchange wait of the pivoted Cholesky timed out");
    }
    hipLaunchKernelGGL(k_chol_uinv_big, dim3(n), dim3(256), 0, st, n, rank, piv, Lg, U, ldu);
    HIPCK(hipGetLastError());
    return true;
  }
  scr.ensure(sizeof(z64) * ((size_t)n * n + (size_t)n * kPb));
  z64* Lg = scr.as<z64>();
  z64* P = Lg + (size_t)n * n;
  hipLaunchKernelGGL(k_pchol_big, dim3(1), dim3(512), 0, st, n, G, ldg, tol, piv, rank, Lg, P, pivot ? 1 : 0);
  HIPCK(hipGetLastError());
  hipLaunchKernelGGL(k_chol_uinv_big, dim3(n), dim3(256), 0, st, n, rank, piv, Lg, U, ldu);
  HIPCK(hipGetLastError());
  return true;
}

}  // namespace eahp
