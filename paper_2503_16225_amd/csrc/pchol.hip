// Diagonally pivoted Cholesky factorisation with rank cut-off and the inverse
// of the factor, for the rank-revealing orthonormalisation of the block FOM
// (CholQR on the Gram matrix of a block): G[piv, piv] = L L^H, pivots below
// tol times the first one end the factorisation (rank r), and the output is
// U = P L^-H (n x r; row piv[k] of U holds row k of L^-H), so that R U has
// orthonormal columns spanning the retained directions of R.
//
// One work-group of 1024 threads, n <= 128, the matrix in registers (thread t
// owns row t/8 and the 16 columns congruent to t mod 8).  Pivoting is logical
// (rows and columns are marked done instead of being exchanged).  The
// triangular inverse runs row by row in pivot order with the 16 columns of
// each row accumulated in the same registers.
#include "devcommon.h"
#include "kernels.h"

namespace eahp {

namespace {
constexpr int kPcMax = 128;
__device__ __forceinline__ z64 cmulz(z64 a, z64 b) { return mk<double>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
}  // namespace

__global__ void __launch_bounds__(1024) k_pchol_reg(int n, const z64* __restrict__ G, int64_t ldg, double tol,
                                                    int* __restrict__ piv, int* __restrict__ rank_out,
                                                    z64* __restrict__ U, int64_t ldu, z64* __restrict__ Lg) {
  __shared__ double diag[kPcMax];
  __shared__ int done[kPcMax];
  __shared__ int pv[kPcMax];
  __shared__ z64 lcol[2][kPcMax];
  __shared__ int sb[2];
  __shared__ int srank;
  __shared__ double sd0;
  const int t = threadIdx.x;
  const int rr = t >> 3, cg = t & 7;
  z64 a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = cg + 8 * m;
    z64 v = mk<double>(0.0, 0.0);
    if (rr < n && c < n) {
      const z64 x = G[rr + (int64_t)c * ldg], y = G[c + (int64_t)rr * ldg];
      v = mk<double>(0.5 * (x.x + y.x), rr == c ? 0.0 : 0.5 * (x.y - y.y));
    }
    a[m] = v;
  }
  if (t < n) {
    diag[t] = G[t + (int64_t)t * ldg].x;
    done[t] = 0;
  }
  if (t == 0) srank = n;
  __syncthreads();
  int r = n;
  for (int k = 0; k < n; ++k) {
    // pivot: largest remaining diagonal (ties: smallest index), wave 0
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = t; i < n; i += 64)
        if (!done[i] && diag[i] > best) {
          best = diag[i];
          bi = i;
        }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (t == 0) {
        if (k == 0) sd0 = best;
        const double d0 = k == 0 ? best : sd0;
        if (!(best > tol * d0) || !(best > 0.0)) srank = k;
        else {
          sb[k & 1] = bi;
          pv[k] = bi;
        }
      }
    }
    __syncthreads();
    if (srank == k) {
      r = k;
      break;
    }
    const int b = sb[k & 1];
    const double lbb = sqrt(diag[b]);
    // column b of the factor: l_i = a_ib / l_bb for the remaining rows, l_b = l_bb
    if (rr < n) {
#pragma unroll
      for (int m = 0; m < 16; ++m)
        if (cg + 8 * m == b) {
          z64 v;
          if (rr == b) v = mk<double>(lbb, 0.0);
          else if (done[rr]) v = mk<double>(0.0, 0.0);
          else v = cscale<double>(a[m], 1.0 / lbb);
          lcol[k & 1][rr] = v;
          Lg[rr + (int64_t)k * n] = v;
          if (rr == b) done[b] = 1;  // read only after the barrier below
        }
    }
    __syncthreads();
    if (rr < n && !done[rr]) {
      const z64 li = lcol[k & 1][rr];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int c = cg + 8 * m;
        if (c < n && !done[c]) {
          const z64 lc = lcol[k & 1][c];
          a[m] = csub<double>(a[m], cmulz(li, mk<double>(lc.x, -lc.y)));
        }
      }
      if (cg == 0) diag[rr] -= li.x * li.x + li.y * li.y;
    }
    __syncthreads();
  }
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
  // X = Lt^-1 with Lt[a][m] = Lg[pv[a] + m n] (lower triangular in pivot order);
  // thread row rr = pivot position, acc[m] = X[rr][cg + 8 m] once row rr is final
  z64 acc[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) acc[m] = mk<double>(0.0, 0.0);
  z64* xrow = &lcol[0][0];  // reused: 2 x kPcMax
  // Lt[rr][arow] is loaded one row ahead so that its latency overlaps the barrier
  z64 lnext = (rr < r) ? Lg[pv[rr]] : mk<double>(0.0, 0.0);
  for (int arow = 0; arow < r; ++arow) {
    z64* xr = xrow + (arow & 1) * kPcMax;
    const z64 l = lnext;
    if (rr < r && arow + 1 < r) lnext = Lg[pv[rr] + (int64_t)(arow + 1) * n];
    if (rr == arow) {
      const double inv = 1.0 / l.x;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int j = cg + 8 * m;
        if (j <= arow) {
          const z64 rhs = csub<double>(mk<double>(j == arow ? 1.0 : 0.0, 0.0), acc[m]);
          acc[m] = cscale<double>(rhs, inv);
          xr[j] = acc[m];
        }
      }
    }
    __syncthreads();
    if (rr > arow && rr < r) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int j = cg + 8 * m;
        if (j <= arow) acc[m] = cadd<double>(acc[m], cmulz(l, xr[j]));
      }
    }
  }
  // U[pv[k]][j] = conj(X[j][k]) for k <= j < r, zero for every other row of column j
  if (rr < r) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int k = cg + 8 * m;
      if (k < n) U[pv[k] + (int64_t)rr * ldu] = k <= rr ? mk<double>(acc[m].x, -acc[m].y) : mk<double>(0.0, 0.0);
    }
  }
}

bool pchol_inv_reg(hipStream_t st, int n, const z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* U,
                   int64_t ldu, DevMem& scr) {
  if (n < 1 || n > kPcMax) return false;
  scr.ensure(sizeof(z64) * (size_t)n * n);
  hipLaunchKernelGGL(k_pchol_reg, dim3(1), dim3(1024), 0, st, n, G, ldg, tol, piv, rank, U, ldu, scr.as<z64>());
  HIPCK(hipGetLastError());
  return true;
}

}  // namespace eahp
