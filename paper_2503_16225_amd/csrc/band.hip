// Projected Sylvester solve of the block FOM (Algorithm 4) for large projected
// systems: (A - s_l I) y_l = c_l for every column l of the right-hand side,
// A (q x q) Hermitian, q > 512.
//
// A is reduced to Hermitian band form B = Q^H A Q of bandwidth kBw by blocked
// Householder transformations (the first stage of a two-stage
// tridiagonalisation).  For every panel of kBw columns:
//   * the block below the band, P (m x kBw), is factored P = H [R; 0] with
//     H = H_0 ... H_{kBw-1}, H_i = I - beta_i v_i v_i^H (a cooperative kernel:
//     one exchange of partial sums between the work-groups per column);
//   * the trailing matrix A22 (m x m) becomes H^H A22 H through the compact
//     WY form H = I - V T V^H, as complex products on the matrix cores:
//       X = A22 V,  Y = X T,  Z = Y - 1/2 V (T^H V^H Y),
//       A22 <- A22 - V Z^H - Z V^H.
// Every shifted system is then a banded solve with partial pivoting, one
// work-group per shift, its active rows in registers:
//   y_l = Q (B - s_l I)^-1 Q^H c_l,
// with Q^H and Q applied as blocked reflector products.  The result is the
// Galerkin solution of the projected equation, the same as through a
// tridiagonal reduction or an eigendecomposition of A (it is unique); the
// O(q^3) part of the work runs as matrix products instead of a matrix-vector
// product with the whole trailing matrix per column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "devcommon.h"
#include "exchange.h"
#include "kernels.h"
#include "ops.h"

namespace eahp {

namespace {
constexpr int kBw = 64;             // bandwidth = panel width (one column per lane)
constexpr int kRw = 2 * kBw + 1;    // stored entries per row of B
constexpr int kWs = kBw + 1;        // active rows of the banded elimination
constexpr int kPanelRpt = 8;        // panel rows per thread (128 rows per work-group)
constexpr int kPanelRows = 16 * kPanelRpt;
constexpr size_t kUbufMax = size_t(8) << 30;  // bytes of eliminated rows held at once
}  // namespace

__global__ void k_band_fill(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Householder QR of the panel P (m x kBw, ld ldp) below the band.  Work-group
// g holds rows g * kPanelRows .. in registers: lane j of wave w has column j
// of rows g * kPanelRows + w + 16 s.  Step i (column i, rows i..m-1):
//   D_j = x^H p_j over rows >= i, x = column i (one exchange of per-group
//   partial sums, added in a fixed order: every work-group gets the same
//   values), r_j = p_{i,j} (row i, held by work-group 0);
//   alpha = -(x_i/|x_i|) ||x||, v = x - alpha e_i, beta = 2 / v^H v,
//   w_j = beta v^H p_j = beta (D_j - conj(alpha) r_j), p_j -= v w_j.
// The lanes m < i of the same sums give v_m^H v_i = conj(D_m) - alpha
// conj(p_{i,m}) (column m holds v_m below its diagonal), the entries of
// G = V^H V, from which work-group 0 forms the compact WY factor
// H_0 ... H_{kBw-1} = I - V T V^H column by column:
//   T_jj = beta_j,  T[0:j, j] = -beta_j T[0:j, 0:j] G[0:j, j].
// Outputs: R (upper triangle) over the first rows of P, v_i (zero above row
// i, v_i[i] = x_i - alpha) into columns 0..kBw-1 and 2kBw..3kBw-1 of V3 and
// into Vh, beta_i, T (kBw x kBw).  A timed-out exchange sets err.
template <int RPT>
__global__ void __launch_bounds__(1024) k_band_panel(int m, z64* P, int64_t ldp, z64* V3, int64_t ldv3, z64* Vh,
                                                     int64_t ldvh, double* beta, z64* Tout, z64* part, z64* rowv,
                                                     int* err) {
  __shared__ z64 red[16][64];
  __shared__ z64 red2[16][64];
  __shared__ z64 rsh[64];
  __shared__ z64 v0s[64];
  __shared__ double bsh[64];
  __shared__ z64 tg[kBw * kBw];  // work-group 0: G (strictly upper part), then T in its place
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int rbase = g * 16 * RPT + w;
  if (g == 0)
    for (int e = threadIdx.x; e < kBw * kBw; e += 1024) tg[e] = mk<double>(0.0, 0.0);
  if (threadIdx.x < kBw) bsh[threadIdx.x] = 0.0;  // columns without a reflector keep beta = 0
  z64 a[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = rbase + 16 * s;
    a[s] = r < m ? P[r + (int64_t)lane * ldp] : mk<double>(0.0, 0.0);
  }
  bool ok = true;
  const int ns = min(kBw, m);
  for (int i = 0; i < ns; ++i) {
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = rbase + 16 * s;
      double xr = readlane_f64(a[s].x, i), xi = readlane_f64(a[s].y, i);
      if (r < i) xr = xi = 0.0;
      ax += xr * a[s].x + xi * a[s].y;  // conj(x) p
      ay += xr * a[s].y - xi * a[s].x;
    }
    red[w][lane] = mk<double>(ax, ay);
    __syncthreads();
    if (w == 0) {
      z64 t = red[0][lane];
      for (int ww = 1; ww < 16; ++ww) t = cadd<double>(t, red[ww][lane]);
      xch::put_z(part + ((int64_t)i * G + g) * 64 + lane, t);
    }
    if (g == 0 && w == (i & 15)) {  // row i: work-group 0, wave i % 16, slot i / 16
#pragma unroll
      for (int s = 0; s < 4 && s < RPT; ++s)
        if (s == (i >> 4)) xch::put_z(rowv + (int64_t)i * 64 + lane, a[s]);
    }
    // wave w adds the partials of work-groups w, w + 16, ... in order (polled
    // four at a time)
    z64 pp = mk<double>(0.0, 0.0);
    const int cnt = w < G ? (G - 1 - w) / 16 + 1 : 0;
    for (int j0 = 0; j0 < cnt; j0 += 4) {
      z64 pv[4];
      const int nn = min(4, cnt - j0);
      xch::poll_zn<4>(part + ((int64_t)i * G + w + 16 * j0) * 64 + lane, 16 * 64, nn, pv, ok);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nn) pp = cadd<double>(pp, pv[j]);
    }
    red2[w][lane] = pp;
    if (w == 15) rsh[lane] = xch::poll_z(rowv + (int64_t)i * 64 + lane, ok);
    __syncthreads();
    z64 D = red2[0][lane];
    for (int ww = 1; ww < 16; ++ww) D = cadd<double>(D, red2[ww][lane]);
    const z64 rj = rsh[lane];
    const double xn2 = fmax(readlane_f64(D.x, i), 0.0);
    const z64 x0 = rsh[i];
    const double xn = sqrt(xn2);
    const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    const z64 alpha = a0 > 0 ? mk<double>(-x0.x / a0 * xn, -x0.y / a0 * xn) : mk<double>(-xn, 0.0);
    const z64 v0 = csub<double>(x0, alpha);
    const double vv = (xn2 - a0 * a0) + (v0.x * v0.x + v0.y * v0.y);
    const double b = vv > 0 ? 2.0 / vv : 0.0;
    const z64 ca = cjmul<double>(alpha, rj);  // conj(alpha) r_j
    const z64 wj = mk<double>(b * (D.x - ca.x), b * (D.y - ca.y));
    if (g == 0 && w == 0 && lane < i) {
      // G[m][i] = v_m^H v_i = conj(D_m) - alpha conj(r_m), m = lane
      const z64 ar = cmul<double>(alpha, mk<double>(rj.x, -rj.y));
      tg[lane + kBw * i] = mk<double>(D.x - ar.x, -D.y - ar.y);
    }
    if (lane > i) {
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = rbase + 16 * s;
        const z64 xv = mk<double>(readlane_f64(a[s].x, i), readlane_f64(a[s].y, i));
        if (r > i) a[s] = csub<double>(a[s], cmul<double>(xv, wj));
        else if (r == i) a[s] = csub<double>(a[s], cmul<double>(v0, wj));
      }
    } else if (lane == i) {
#pragma unroll
      for (int s = 0; s < RPT; ++s)
        if (rbase + 16 * s == i) a[s] = alpha;
    }
    if (threadIdx.x == 0) {
      v0s[i] = v0;
      bsh[i] = b;
    }
  }
  __syncthreads();
  if (!ok) err[0] = 1;
  if (g == 0) {
    // T column by column, in place of G: lane l of wave pp adds the terms
    // m = l + pp, l + pp + 16, ... of sum_m T[l][m] G[m][j]; the 16 partial
    // sums are added in order
    for (int j = 0; j < kBw; ++j) {
      z64 acc = mk<double>(0.0, 0.0);
      for (int mm = lane + w; mm < j; mm += 16) acc = cadd<double>(acc, cmul<double>(tg[lane + kBw * mm], tg[mm + kBw * j]));
      red[w][lane] = acc;
      __syncthreads();
      if (w == 0) {
        z64 tot = red[0][lane];
        for (int ww = 1; ww < 16; ++ww) tot = cadd<double>(tot, red[ww][lane]);
        const double bj = bsh[j];
        tg[lane + kBw * j] = lane < j ? mk<double>(-bj * tot.x, -bj * tot.y)
                                      : (lane == j ? mk<double>(bj, 0.0) : mk<double>(0.0, 0.0));
      }
      __syncthreads();
    }
    for (int e = threadIdx.x; e < kBw * kBw; e += 1024) Tout[e] = tg[e];
  }
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = rbase + 16 * s, j = lane;
    if (r >= m) continue;
    if (r <= j) P[r + (int64_t)j * ldp] = a[s];
    const z64 vj = (j >= ns || r < j) ? mk<double>(0.0, 0.0) : (r == j ? v0s[j] : a[s]);
    V3[r + (int64_t)j * ldv3] = vj;
    V3[r + (int64_t)(2 * kBw + j) * ldv3] = vj;
    Vh[r + (int64_t)j * ldvh] = vj;
  }
  if (g == 0 && threadIdx.x < kBw) beta[threadIdx.x] = (int)threadIdx.x < ns ? bsh[threadIdx.x] : 0.0;
}

// The block update between two panels, W = (I - V T V^H)^H-side terms of
// A22 <- H^H A22 H with H = I - V T V^H and X = A22 V (Hermitian A22):
//   Y = X T,  N = V^H Y,  M = T^H N,  Z = Y - V M / 2,
//   A22 -= V Z^H + Z V^H  (the next panel's columns here, the rest later).
// Three launches for what are otherwise five products and their split-K
// reductions; every sum runs in a fixed order.  Blocks of 64 rows; in LDS a
// 64 x 64 block is row-major with a stride of 65.
constexpr int kWyLd = kBw + 1;
// a conj(b)
__device__ __forceinline__ z64 mulc(z64 a, z64 b) { return mk<double>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }

// k_wy_y: one work-group per 64 rows b: Y_b = X_b T (written to Y) and the
// partial N_b = V_b^H Y_b (to Np[b], 64 x 64 column-major).  Thread t takes
// row (or column) t % 64 and the 4 columns t / 64 + 16 j.
__global__ void __launch_bounds__(1024) k_wy_y(int m, const z64* __restrict__ X, int64_t ldx, const z64* __restrict__ T,
                                              const z64* __restrict__ V, int64_t ldv, z64* __restrict__ Y,
                                              int64_t ldy, z64* __restrict__ Np) {
  __shared__ z64 sa[kBw * kWyLd];
  __shared__ z64 sb[kBw * kWyLd];
  const int t = threadIdx.x, r = t & 63, c0 = t >> 6;
  const int64_t rb = (int64_t)blockIdx.x * kBw;
  for (int e = t; e < kBw * kBw; e += 1024) {
    const int i = e & 63, k = e >> 6;
    sa[i * kWyLd + k] = rb + i < m ? X[rb + i + (int64_t)k * ldx] : mk<double>(0.0, 0.0);
    sb[i * kWyLd + k] = T[i + (int64_t)k * kBw];
  }
  __syncthreads();
  z64 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = mk<double>(0.0, 0.0);
  for (int k = 0; k < kBw; ++k) {
    const z64 x = sa[r * kWyLd + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = cadd<double>(acc[j], cmul<double>(x, sb[k * kWyLd + c0 + 16 * j]));
  }
  if (rb + r < m) {
#pragma unroll
    for (int j = 0; j < 4; ++j) Y[rb + r + (int64_t)(c0 + 16 * j) * ldy] = acc[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) sa[r * kWyLd + c0 + 16 * j] = rb + r < m ? acc[j] : mk<double>(0.0, 0.0);
  for (int e = t; e < kBw * kBw; e += 1024) {
    const int i = e & 63, k = e >> 6;
    sb[i * kWyLd + k] = rb + i < m ? V[rb + i + (int64_t)k * ldv] : mk<double>(0.0, 0.0);
  }
  __syncthreads();
  // N_b[c1][c2] = sum_i conj(V[i][c1]) Y[i][c2], c1 = t % 64, c2 = t / 64 + 16 j
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = mk<double>(0.0, 0.0);
  for (int i = 0; i < kBw; ++i) {
    const z64 v = sb[i * kWyLd + r];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = cadd<double>(acc[j], cjmul<double>(v, sa[i * kWyLd + c0 + 16 * j]));
  }
  z64* P = Np + (int64_t)blockIdx.x * kBw * kBw;
#pragma unroll
  for (int j = 0; j < 4; ++j) P[r + (c0 + 16 * j) * kBw] = acc[j];
}

// k_wy_m: one work-group per column c of N: N[:, c] = sum_b Np[b][:, c]
// (four groups of blocks, added in a fixed order), M[:, c] = T^H N[:, c],
// and Z_0[:, c] = Y_0[:, c] - V_0 M[:, c] / 2 for the first 64 rows (written
// over Y), which every work-group of k_wy_z needs.
__global__ void __launch_bounds__(256) k_wy_m(int m, int nb, const z64* __restrict__ Np, const z64* __restrict__ T,
                                              z64* __restrict__ M, const z64* __restrict__ V, int64_t ldv, z64* Y,
                                              int64_t ldy, unsigned long long* fillp, int64_t nfill) {
  // the exchange slots of the next panel back to the empty pattern (the
  // current panel, which used them, has finished)
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nfill; e += (int64_t)gridDim.x * blockDim.x)
    fillp[e] = xch::kEmpty;
  __shared__ z64 big[kBw * kWyLd];
  __shared__ z64 red[4][kBw];
  __shared__ z64 ncol[kBw], mcol[kBw];
  const int t = threadIdx.x, i = t & 63, g = t >> 6;
  const int c = blockIdx.x;
  z64 s = mk<double>(0.0, 0.0);
  for (int bb = g; bb < nb; bb += 4) s = cadd<double>(s, Np[(int64_t)bb * kBw * kBw + i + c * kBw]);
  red[g][i] = s;
  // T into LDS, row-major: big[k][i] = T[k][i]
  for (int e = t; e < kBw * kBw; e += 256) {
    const int k = e & 63, ii = e >> 6;
    big[k * kWyLd + ii] = T[k + (int64_t)ii * kBw];
  }
  __syncthreads();
  if (t < kBw) ncol[t] = cadd<double>(cadd<double>(red[0][t], red[1][t]), cadd<double>(red[2][t], red[3][t]));
  __syncthreads();
  if (t < kBw) {
    // M[t][c] = sum_k conj(T[k][t]) N[k][c]
    z64 a = mk<double>(0.0, 0.0);
    for (int k = 0; k < kBw; ++k) a = cadd<double>(a, cjmul<double>(big[k * kWyLd + t], ncol[k]));
    mcol[t] = a;
    M[t + (int64_t)c * kBw] = a;
  }
  __syncthreads();
  for (int e = t; e < kBw * kBw; e += 256) {
    const int rr = e & 63, k = e >> 6;
    big[rr * kWyLd + k] = rr < m ? V[rr + (int64_t)k * ldv] : mk<double>(0.0, 0.0);
  }
  __syncthreads();
  if (t < kBw && t < m) {
    z64 a = mk<double>(0.0, 0.0);
    for (int k = 0; k < kBw; ++k) a = cadd<double>(a, cmul<double>(big[t * kWyLd + k], mcol[k]));
    z64* y = Y + t + (int64_t)c * ldy;
    *y = mk<double>(y->x - 0.5 * a.x, y->y - 0.5 * a.y);
  }
}

// k_wy_z: one work-group per 64 rows b: Z_b = Y_b - V_b M / 2 (b >= 1; block
// 0 comes from k_wy_m) written over Y, and with upd the next panel's columns
// A22[rows of b, 0:64] -= V_b Z_0^H + Z_b V_0^H.
__global__ void __launch_bounds__(1024) k_wy_z(int m, const z64* __restrict__ M, const z64* __restrict__ V,
                                              int64_t ldv, z64* Y, int64_t ldy, z64* A22, int64_t lda, int upd) {
  __shared__ z64 sa[kBw * kWyLd];
  __shared__ z64 sb[kBw * kWyLd];
  const int t = threadIdx.x, r = t & 63, c0 = t >> 6;
  const int b = blockIdx.x;
  const int64_t rb = (int64_t)b * kBw;
  const bool live = rb + r < m;
  auto load_rows = [&](z64* dst, const z64* src, int64_t ld, int64_t row0) __attribute__((always_inline)) {
    for (int e = t; e < kBw * kBw; e += 1024) {
      const int i = e & 63, k = e >> 6;
      dst[i * kWyLd + k] = row0 + i < m ? src[row0 + i + (int64_t)k * ld] : mk<double>(0.0, 0.0);
    }
  };
  z64 z[4];
  if (b == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) z[j] = live ? Y[r + (int64_t)(c0 + 16 * j) * ldy] : mk<double>(0.0, 0.0);
  } else {
    for (int e = t; e < kBw * kBw; e += 1024) {
      const int k = e & 63, cc = e >> 6;
      sa[k * kWyLd + cc] = M[k + (int64_t)cc * kBw];
    }
    load_rows(sb, V, ldv, rb);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) z[j] = mk<double>(0.0, 0.0);
    for (int k = 0; k < kBw; ++k) {
      const z64 v = sb[r * kWyLd + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) z[j] = cadd<double>(z[j], cmul<double>(v, sa[k * kWyLd + c0 + 16 * j]));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const z64 y = live ? Y[rb + r + (int64_t)(c0 + 16 * j) * ldy] : mk<double>(0.0, 0.0);
      z[j] = mk<double>(y.x - 0.5 * z[j].x, y.y - 0.5 * z[j].y);
    }
    if (live) {
#pragma unroll
      for (int j = 0; j < 4; ++j) Y[rb + r + (int64_t)(c0 + 16 * j) * ldy] = z[j];
    }
  }
  if (!upd) return;  // uniform over the work-group
  // Z_b V_0^H
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) sa[r * kWyLd + c0 + 16 * j] = live ? z[j] : mk<double>(0.0, 0.0);
  load_rows(sb, V, ldv, 0);
  __syncthreads();
  z64 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = mk<double>(0.0, 0.0);
  for (int k = 0; k < kBw; ++k) {
    const z64 zr = sa[r * kWyLd + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = cadd<double>(acc[j], mulc(zr, sb[(c0 + 16 * j) * kWyLd + k]));
  }
  // V_b Z_0^H
  __syncthreads();
  load_rows(sa, V, ldv, rb);
  load_rows(sb, Y, ldy, 0);
  __syncthreads();
  z64 acc1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc1[j] = mk<double>(0.0, 0.0);
  for (int k = 0; k < kBw; ++k) {
    const z64 vr = sa[r * kWyLd + k];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc1[j] = cadd<double>(acc1[j], mulc(vr, sb[(c0 + 16 * j) * kWyLd + k]));
  }
  if (live) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      z64* a = A22 + rb + r + (int64_t)(c0 + 16 * j) * lda;
      const z64 d = cadd<double>(acc1[j], acc[j]);
      *a = mk<double>(a->x - d.x, a->y - d.y);
    }
  }
}

// Rows of the band matrix: RB[r * kRw + t] = B[r][r - kBw + t] (t = 0..2kBw),
// zero outside the matrix; entries on and below the diagonal come from the
// lower triangle of A, the others as conjugates of their mirror.
__global__ void k_band_rows(int q, const z64* __restrict__ A, int64_t lda, z64* __restrict__ RB) {
  const int64_t n = (int64_t)q * kRw;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / kRw), t = (int)(e - (int64_t)r * kRw);
    const int c = r - kBw + t;
    z64 v = mk<double>(0.0, 0.0);
    if (c >= 0 && c < q) {
      if (c <= r) v = A[r + (int64_t)c * lda];
      else {
        const z64 u = A[c + (int64_t)r * lda];
        v = mk<double>(u.x, -u.y);
      }
    }
    RB[e] = v;
  }
}

// Banded solve with partial pivoting, (B - s I) y = c, one shift per
// work-group (shift l0 + blockIdx.x, right-hand side and solution in column
// l0 + blockIdx.x of Y), blocked by panels of kNb columns.
//
// Gaussian elimination with row pivoting picks the pivot of column k among
// the rows not yet eliminated; a row r is zero left of column r - kBw, so the
// pivot lies in rows k .. k + kBw and the pivot row has its non-zeros in
// columns k .. k + 2kBw.  The rows that can take part in the panel of columns
// k0 .. k0 + kNb - 1 are the kBw rows left over from earlier panels and the
// kNb rows k0 + kBw .. k0 + kBw + kNb - 1; they sit in kWin row slots, and a
// row keeps its slot until it becomes a pivot (its slot then takes a row of
// the next panel).  Thread t holds column slot t % 128 of the row slots
// t / 128 + 8 i in registers, over the columns right of the panel (column c
// in slot c % 128); the panel's own columns are moved to LDS.  Per panel:
//   * one wave factors the kWin x kNb panel (pivot search, multipliers
//     L, the panel part of the pivot rows, the right-hand sides) and
//     inverts the unit lower triangle L11 of the pivot rows' multipliers;
//   * the pivot rows' parts right of the panel become U12 = L11^-1 A12;
//   * every other row is updated with the rank-kNb product L21 U12.
// Eliminated rows go to Ubuf (row k: U[k][0] the pivot, U[k][1 + d] the entry
// in column k + 1 + d) and the transformed right-hand side into y; the
// triangular system U y = z is then solved backwards by one wave, its rows
// staged through LDS by the whole work-group.
constexpr int kNb = 8;                                 // columns per panel
constexpr int kWin = kBw + kNb;                        // row slots
constexpr int kGt = 1024;                              // threads per work-group
constexpr int kRpt = kWin / 8;                         // row slots per thread
constexpr int kEnt = kRw + 1;                          // band of an entering row and its right-hand side
constexpr int kEntN = kNb * kEnt;                      // staged values of a panel's entering rows
constexpr int kEntPer = (kEntN + kGt - 1) / kGt;
constexpr int kBsChunk = 8;                            // rows of U per LDS stage in the backward solve
__device__ __forceinline__ z64 zz() { return mk<double>(0.0, 0.0); }

__global__ void __launch_bounds__(kGt) k_band_gepp(int q, const z64* __restrict__ RB,
                                                      const double* __restrict__ shift, z64* __restrict__ Y,
                                                      int64_t ldy, z64* __restrict__ Ubuf, int l0) {
  __shared__ z64 pnl[kWin][kNb + 1];  // the panel's columns of every slot; multipliers after the panel step
  __shared__ z64 big[kEntN];          // entering rows, then A12 / U12 (kNb x 128)
  __shared__ z64 ust[2][kBsChunk][kEnt];  // backward solve: rows of U and z
  __shared__ z64 linv[kNb][kNb + 1];  // inverse of L11
  __shared__ z64 rhs[kWin];
  __shared__ int rid[kWin];  // row held by each slot (-1: none)
  __shared__ int piv[kWin];  // panel column at which the slot's row became the pivot (-1: not yet)
  __shared__ int inc[kWin];  // entering row taken by the slot in this panel (-1: none)
  __shared__ int pj[kNb];    // slot of the pivot of each panel column
  __shared__ int freel[kNb]; // slots freed by the last panel
  __shared__ z64 wsave[kRpt][64];  // wave 0's window slots during the panel
  const int l = l0 + blockIdx.x;
  const double sft = shift[l];
  z64* y = Y + (int64_t)l * ldy;
  z64* U = Ubuf + (int64_t)blockIdx.x * q * kRw;
  const int t = threadIdx.x, cs = t & 127, rg = t >> 7, lane = t & 63, wv = t >> 6;
  auto bval = [&](int r, int c) __attribute__((always_inline)) -> z64 {
    if (r >= q || c < 0 || c >= q || c < r - kBw || c > r + kBw) return zz();
    z64 v = RB[(int64_t)r * kRw + (c - r + kBw)];
    if (r == c) v.x -= sft;
    return v;
  };
  // value e of the rows entering the panel at k0: row i = e / kEnt, entry d
  // (d < kRw: B - s I at column r - kBw + d; d = kRw: the right-hand side)
  auto ent_val = [&](int k0, int e) __attribute__((always_inline)) -> z64 {
    if (e >= kEntN) return zz();
    const int i = e / kEnt, d = e - i * kEnt;
    const int r = k0 + kBw + i;
    if (r >= q) return zz();
    if (d == kRw) return y[r];
    if (r - kBw + d >= q) return zz();
    z64 v = RB[(int64_t)r * kRw + d];
    if (d == kBw) v.x -= sft;
    return v;
  };
  z64 w[kRpt];  // row slots rg + 8 i, column slot cs
  z64 pre[kEntPer];
#pragma unroll
  for (int i = 0; i < kRpt; ++i) {
    const int sl = rg + 8 * i;
    w[i] = sl < kBw ? bval(sl, cs) : zz();  // rows 0..kBw-1, columns 0..127
  }
  if (t < kWin) {
    rid[t] = (t < kBw && t < q) ? t : -1;
    rhs[t] = (t < kBw && t < q) ? y[t] : zz();
  }
  if (t < kNb) freel[t] = kBw + t;
#pragma unroll
  for (int u = 0; u < kEntPer; ++u) pre[u] = ent_val(0, t + kGt * u);
  __syncthreads();
  for (int k0 = 0; k0 < q; k0 += kNb) {
    const int nsk = min(kNb, q - k0);
    // (1) the entering rows into LDS (the next panel's are prefetched); the
    // panel's columns to LDS, their register slots now hold columns
    // k0 + 128 .. k0 + 143 (zero in every row left over)
#pragma unroll
    for (int u = 0; u < kEntPer; ++u) {
      const int e = t + kGt * u;
      if (e < kEntN) big[e] = pre[u];
    }
#pragma unroll
    for (int u = 0; u < kEntPer; ++u) pre[u] = ent_val(k0 + kNb, t + kGt * u);
    const int jc = (cs - k0) & 127;
    if (jc < kNb) {
#pragma unroll
      for (int i = 0; i < kRpt; ++i) {
        pnl[rg + 8 * i][jc] = w[i];
        w[i] = zz();
      }
    }
    if (t < kWin) {
      int ii = -1;
      for (int i = 0; i < kNb; ++i)
        if (freel[i] == t) ii = i;
      inc[t] = ii;
      piv[t] = -1;
    }
    __syncthreads();
    // (2) the entering rows into the freed slots
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
      const int sl = rg + 8 * i, ii = inc[sl];
      if (ii >= 0) {
        const int d = kNb + ((cs - k0 - kNb) & 127) - ii;  // column k0 + kNb + ((cs - k0 - kNb) mod 128)
        w[i] = d <= 2 * kBw ? big[ii * kEnt + d] : zz();
        if (cs < kNb) pnl[sl][cs] = cs >= ii ? big[ii * kEnt + cs - ii] : zz();
      }
    }
    if (t < kWin && inc[t] >= 0) {
      const int ii = inc[t], r = k0 + kBw + ii;
      rhs[t] = big[ii * kEnt + kRw];
      rid[t] = r < q ? r : -1;
    }
    __syncthreads();
    // (3) the panel, by wave 0, in registers: lane j holds slots j and j + 64
    // (j < kNb); the pivot row is broadcast from its lane.  Wave 0 parks its
    // window slots in LDS meanwhile (the branch is uniform, so they take no
    // registers inside it).
    if (__builtin_amdgcn_readfirstlane(wv) == 0) {
#pragma unroll
      for (int i = 0; i < kRpt; ++i) wsave[i][lane] = w[i];
      const int s0 = lane, s1 = lane + 64;
      const bool has1 = lane < kWin - 64;
      z64 r0[kNb], r1[kNb];
#pragma unroll
      for (int cc = 0; cc < kNb; ++cc) {
        r0[cc] = pnl[s0][cc];
        r1[cc] = has1 ? pnl[s1][cc] : zz();
      }
      bool act0 = rid[s0] >= 0, act1 = has1 && rid[s1] >= 0;
      z64 h0 = rhs[s0], h1 = has1 ? rhs[s1] : zz();
#pragma unroll
      for (int j = 0; j < kNb; ++j) {
        if (j < nsk) {
          double v = act0 ? r0[j].x * r0[j].x + r0[j].y * r0[j].y : -1.0;
          int ix = s0;
          argmax_merge(v, ix, act1 ? r1[j].x * r1[j].x + r1[j].y * r1[j].y : -1.0, s1);
          wave_argmax(v, ix);
          const int p = ix, pl = p & 63;
          const bool ph = p >= 64;
          z64 prow[kNb];
#pragma unroll
          for (int cc = 0; cc < kNb; ++cc) {
            if (cc >= j) {
              const z64 src = ph ? r1[cc] : r0[cc];
              prow[cc] = mk<double>(readlane_f64(src.x, pl), readlane_f64(src.y, pl));
            }
          }
          const z64 hs = ph ? h1 : h0;
          const z64 zp = mk<double>(readlane_f64(hs.x, pl), readlane_f64(hs.y, pl));
          const double rd = 1.0 / (prow[j].x * prow[j].x + prow[j].y * prow[j].y);
          const z64 inv = mk<double>(prow[j].x * rd, -prow[j].y * rd);
          if (act0 && s0 != p) {
            const z64 lr = cmul<double>(r0[j], inv);
            r0[j] = lr;
#pragma unroll
            for (int cc = 0; cc < kNb; ++cc)
              if (cc > j) r0[cc] = csub<double>(r0[cc], cmul<double>(lr, prow[cc]));
            h0 = csub<double>(h0, cmul<double>(lr, zp));
          }
          if (act1 && s1 != p) {
            const z64 lr = cmul<double>(r1[j], inv);
            r1[j] = lr;
#pragma unroll
            for (int cc = 0; cc < kNb; ++cc)
              if (cc > j) r1[cc] = csub<double>(r1[cc], cmul<double>(lr, prow[cc]));
            h1 = csub<double>(h1, cmul<double>(lr, zp));
          }
          if (s0 == p) {
            act0 = false;
            piv[s0] = j;
          }
          if (s1 == p) {
            act1 = false;
            piv[s1] = j;
          }
          if (lane == 0) pj[j] = p;
        }
      }
#pragma unroll
      for (int cc = 0; cc < kNb; ++cc) {
        pnl[s0][cc] = r0[cc];
        if (has1) pnl[s1][cc] = r1[cc];
      }
      rhs[s0] = h0;
      if (has1) rhs[s1] = h1;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // L11^-1, column i by lane i: X[i][i] = 1, X[j][i] = -sum_{m=i..j-1} L[j][m] X[m][i]
      if (lane < kNb) {
        const int i = lane;
        for (int j = 0; j < kNb; ++j) {
          z64 x = zz();
          if (j == i) x = mk<double>(1.0, 0.0);
          else if (j > i && j < nsk) {
            const int pr = pj[j];
            for (int m = i; m < j; ++m) x = csub<double>(x, cmul<double>(pnl[pr][m], linv[m][i]));
          }
          linv[j][i] = x;
        }
      }
#pragma unroll
      for (int i = 0; i < kRpt; ++i) w[i] = wsave[i][lane];
    }
    __syncthreads();
    // (4) the pivot rows right of the panel (A12) into LDS
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
      const int jj = piv[rg + 8 * i];
      if (jj >= 0) big[jj * 128 + cs] = w[i];
    }
    __syncthreads();
    // (5) U12 = L11^-1 A12: thread (rg, cs) forms row rg
    {
      const int j = rg;
      z64 acc = zz();
#pragma unroll
      for (int i = 0; i < kNb; ++i)
        if (i <= j && j < nsk) acc = cadd<double>(acc, cmul<double>(linv[j][i], big[i * 128 + cs]));
      __syncthreads();
      big[j * 128 + cs] = acc;
    }
    __syncthreads();
    // (6) rank-kNb update of the other rows; the pivot rows go to U, their
    // right-hand sides to y, their slots to the next panel
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
      const int sl = rg + 8 * i;
      if (rid[sl] >= 0 && piv[sl] < 0) {
        z64 acc = w[i];
#pragma unroll
        for (int jj = 0; jj < kNb; ++jj)
          if (jj < nsk) acc = csub<double>(acc, cmul<double>(pnl[sl][jj], big[jj * 128 + cs]));
        w[i] = acc;
      }
    }
    for (int e = t; e < kNb * kRw; e += kGt) {
      const int j = e / kRw, dd = e - j * kRw;
      if (j < nsk) {
        const int pr = pj[j], k = k0 + j;
        z64 v;
        if (dd == 0) v = pnl[pr][j];
        else {
          const int c = k + dd;
          v = c < k0 + kNb ? pnl[pr][c - k0] : big[j * 128 + (c & 127)];
        }
        U[(int64_t)k * kRw + dd] = v;
      }
    }
    if (t < nsk) {
      y[k0 + t] = rhs[pj[t]];
      freel[t] = pj[t];
    }
    __syncthreads();
  }
  // ---- backward solve U y = z.  Chunks of kBsChunk rows, from the last:
  // every thread loads its share of the next chunk while wave 0 solves the
  // current one from LDS.  Lane j of wave 0 holds y[k+1+j] and y[k+65+j].
  const int nch = (q + kBsChunk - 1) / kBsChunk;
  constexpr int kPer = kBsChunk * kEnt;
  constexpr int kPerT = (kPer + kGt - 1) / kGt;
  auto stage_ld = [&](int ch, z64* vals) __attribute__((always_inline)) {
    const int r0 = ch * kBsChunk;
#pragma unroll
    for (int u = 0; u < kPerT; ++u) {
      const int e = t + kGt * u;
      z64 v = zz();
      if (e < kPer) {
        const int rr = e / kEnt, cc = e - rr * kEnt;
        const int k = r0 + rr;
        if (k < q) v = cc < kRw ? U[(int64_t)k * kRw + cc] : y[k];
      }
      vals[u] = v;
    }
  };
  auto stage_st = [&](int buf, const z64* vals) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kPerT; ++u) {
      const int e = t + kGt * u;
      if (e < kPer) (&ust[buf][0][0])[e] = vals[u];
    }
  };
  z64 sv[kPerT];
  stage_ld(nch - 1, sv);
  stage_st((nch - 1) & 1, sv);
  __syncthreads();
  z64 ya = zz(), yb = zz();
  for (int ch = nch - 1; ch >= 0; --ch) {
    if (ch > 0) stage_ld(ch - 1, sv);
    if (t < 64) {
      const int r0 = ch * kBsChunk;
      const int rr_hi = min(kBsChunk, q - r0) - 1;
      for (int rr = rr_hi; rr >= 0; --rr) {
        const z64* Ur = ust[ch & 1][rr];
        const z64 ua = Ur[1 + t], ub = Ur[1 + kBw + t], u0 = Ur[0], zk = Ur[kRw];
        double sx = ua.x * ya.x - ua.y * ya.y + ub.x * yb.x - ub.y * yb.y;
        double sy = ua.x * ya.y + ua.y * ya.x + ub.x * yb.y + ub.y * yb.x;
        sx = wave_allsum(sx);
        sy = wave_allsum(sy);
        const double nx = zk.x - sx, ny = zk.y - sy;
        const double rd = 1.0 / (u0.x * u0.x + u0.y * u0.y);
        const z64 yk = mk<double>((nx * u0.x + ny * u0.y) * rd, (ny * u0.x - nx * u0.y) * rd);
        if (t == 0) y[r0 + rr] = yk;
        const double a63x = __shfl(ya.x, 63, 64), a63y = __shfl(ya.y, 63, 64);
        const double uax = __shfl_up(ya.x, 1, 64), uay = __shfl_up(ya.y, 1, 64);
        const double ubx = __shfl_up(yb.x, 1, 64), uby = __shfl_up(yb.y, 1, 64);
        ya = t == 0 ? yk : mk<double>(uax, uay);
        yb = t == 0 ? mk<double>(a63x, a63y) : mk<double>(ubx, uby);
      }
    }
    if (ch > 0) stage_st((ch - 1) & 1, sv);
    __syncthreads();
  }
}

// The projected solve for q > kBw (the FOM calls it beyond q = 512): A (q x q,
// ld lda, Hermitian up to rounding; destroyed), s (p shifts), Yt (q x p, ld q:
// the right-hand sides, overwritten by the solutions).
void sylvester_band(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws,
                    DevMem& part, const BandAux* aux) {
  if (q <= kBw) fail(EAHP_EINVAL, "band reduction: q must exceed the bandwidth");
  if (p <= 0) return;
  const int b = kBw;
  int dev = 0, ncu = 0;
  HIPCK(hipGetDevice(&dev));
  HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int gmax = (q - b + kPanelRows - 1) / kPanelRows;
  if (gmax > ncu) fail(EAHP_EINVAL, "band reduction: projected system too large for one cooperative panel");
  // shifts per elimination launch: the eliminated rows of each are kept
  const size_t ubytes_shift = sizeof(z64) * (size_t)q * kRw;
  const int nsh = (int)std::max<size_t>(1, std::min<size_t>((size_t)p, kUbufMax / ubytes_shift));
  // workspace: Vh (q x q), beta (q), V3 (q x 3b), X (q x b), T, N, M (b x b),
  // RB (q x kRw), exchange slots, error flag, blocked-product scratch, U rows
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t oVh = 0;
  const size_t oBt = oVh + al(sizeof(z64) * (size_t)q * q);
  const size_t oV3 = oBt + al(sizeof(double) * q);
  const size_t oX = oV3 + al(sizeof(z64) * (size_t)q * 3 * b * 2);  // two buffers (look-ahead)
  const size_t oSm = oX + al(sizeof(z64) * (size_t)q * b);
  const size_t oRB = oSm + al(sizeof(z64) * 3 * b * b);
  const size_t oSl = oRB + al(sizeof(z64) * (size_t)q * kRw);
  const size_t nslot = (size_t)b * (gmax + 1) * 64;
  const size_t oErr = oSl + al(sizeof(z64) * nslot);
  const int npan = (q - b + b - 1) / b;  // panels (k0 = 0, b, ... while k0 + b < q)
  const size_t oTa = oErr + 256;       // the compact WY factor T of every panel
  const size_t oZf = oTa + al(sizeof(z64) * (size_t)npan * b * b);  // V^H C~ and T^H V^H C~ (b x p each)
  const size_t oNp = oZf + al(sizeof(z64) * 2 * (size_t)b * p);  // partial N of the block update: one 64 x 64 block per 64 rows
  const size_t oWy = oNp + al(sizeof(z64) * (size_t)((q + kBw - 1) / kBw) * kBw * kBw);
  const size_t oU = oWy + al(refl_blocked_scratch(q - b, p));
  ws.ensure(oU + ubytes_shift * nsh);
  char* base = static_cast<char*>(ws.p);
  z64* Vh = reinterpret_cast<z64*>(base + oVh);
  double* bt = reinterpret_cast<double*>(base + oBt);
  z64* V3 = reinterpret_cast<z64*>(base + oV3);
  z64* X = reinterpret_cast<z64*>(base + oX);
  z64* Tm = reinterpret_cast<z64*>(base + oSm);
  z64* Nm = Tm + b * b;
  z64* Mm = Nm + b * b;
  z64* RB = reinterpret_cast<z64*>(base + oRB);
  z64* slots = reinterpret_cast<z64*>(base + oSl);
  int* err = reinterpret_cast<int*>(base + oErr);
  void* wy = base + oWy;
  z64* Npart = reinterpret_cast<z64*>(base + oNp);
  z64* Tall = reinterpret_cast<z64*>(base + oTa);
  z64* Zf = reinterpret_cast<z64*>(base + oZf);
  z64* Zf2 = Zf + (size_t)b * p;
  z64* Ubuf = reinterpret_cast<z64*>(base + oU);
  const int64_t ld3 = q;

  hermitize(st, q, A, lda, 0, 1);
  {
    const int64_t nw = (int64_t)2 * q * q;
    hipLaunchKernelGGL(k_band_fill, dim3((unsigned)std::min<int64_t>(4096, (nw + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<unsigned long long*>(Vh), nw, 0ull);
    hipLaunchKernelGGL(k_band_fill, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned long long*>(err), (int64_t)1,
                       0ull);
  }
  {
    // the cooperative panels wait on each other's work-groups: one such grid
    // at a time per process
    std::lock_guard<std::mutex> lk(coop_mutex());
    // With look-ahead, panel i's update of the trailing matrix beyond the
    // next panel's columns runs on the second stream while panel i + 1 is
    // factored: the next panel's columns are updated first, and panel i + 1
    // reads and writes only those columns; X of panel i + 1 waits for the
    // rest.  That update is submitted after panel i + 1, so that the panel's
    // work-groups (which wait on each other) are dispatched first.  V3
    // alternates between two buffers (the second stream still reads panel
    // i's while panel i + 1 writes its own).
    const bool look = aux != nullptr && aux->s != nullptr;
    // With the second stream, panel i's reflectors are also applied to the
    // right-hand sides there (C~ <- P_i^H C~ with P_i = I - V_i T_i V_i^H,
    // V_i from Vh, T_i kept per panel), behind panel i's trailing update, so
    // that this work fills the CUs the latency-bound panels leave idle; the
    // blocked forward application after the reduction is then skipped.
    const bool fwd_on_aux = look && aux->part != nullptr && aux->f != nullptr;
    struct Deferred {
      bool on = false, upd = false;
      int m = 0, k0 = 0, ns = 0, idx = 0;
      z64 *V3 = nullptr, *Yb = nullptr, *A22 = nullptr;
    } rest;
    auto submit_rest = [&]() {
      HIPCK(hipStreamWaitEvent(aux->s, aux->z, 0));
      if (rest.upd) {
        // A22[:, b:] -= [V Z] [Z V]^H[:, b:] on the second stream, after the event z
        gemm_nn<double>(aux->s, rest.m, 2 * b, rest.m - b, rest.V3, ld3, rest.Yb + b, ld3, 1,
                        rest.A22 + (int64_t)b * lda, lda, -1.0, 0.0, 1.0);
        HIPCK(hipEventRecord(aux->c, aux->s));
      }
      if (fwd_on_aux) {
        const int r0 = rest.k0 + b;
        const z64* Vi = Vh + (int64_t)rest.k0 * q + r0;
        const z64* Ti = Tall + (int64_t)rest.idx * b * b;
        gemm_hn<double>(aux->s, rest.m, rest.ns, p, Vi, q, Yt + r0, q, Zf, rest.ns, 1.0, 0.0, *aux->part);
        gemm_hn<double>(aux->s, rest.ns, rest.ns, p, Ti, b, Zf, rest.ns, Zf2, rest.ns, 1.0, 0.0, *aux->part);
        gemm_nn<double>(aux->s, rest.m, rest.ns, p, Vi, q, Zf2, rest.ns, 0, Yt + r0, q, -1.0, 0.0, 1.0);
        HIPCK(hipEventRecord(aux->f, aux->s));
      }
      rest.on = false;
      return true;
    };
    for (int k0 = 0, idx = 0; k0 + b < q; k0 += b, ++idx) {
      const int m = q - k0 - b, ns = std::min(b, m);
      const int G = (m + kPanelRows - 1) / kPanelRows;
      z64* P = A + (k0 + b) + (int64_t)k0 * lda;
      z64* V3c = V3 + (int64_t)(idx & 1) * ld3 * 3 * b;
      z64* part_x = slots;
      z64* rowv = slots + (size_t)ns * G * 64;
      // the first panel's exchange slots here; the later ones' by k_wy_m of the panel before
      if (idx == 0) {
        const int64_t nw = (int64_t)2 * ns * (G + 1) * 64;
        hipLaunchKernelGGL(k_band_fill, dim3((unsigned)std::min<int64_t>(1024, (nw + 255) / 256)), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long*>(slots), nw, xch::kEmpty);
      }
      int mm = m;
      int64_t ldp = lda, ldv = ld3, ldh = q;
      z64* Vp = Vh + (int64_t)k0 * q + (k0 + b);
      double* btp = bt + k0;
      z64* Tp = Tall + (int64_t)idx * b * b;
      void* args[] = {&mm, &P, &ldp, &V3c, &ldv, &Vp, &ldh, &btp, &Tp, &part_x, &rowv, &err};
      HIPCK(hipLaunchCooperativeKernel((const void*)k_band_panel<kPanelRpt>, dim3(G), dim3(1024), args, 0, st));
      if (rest.on) {
        const bool had_upd = rest.upd;
        submit_rest();
        if (had_upd) HIPCK(hipStreamWaitEvent(st, aux->c, 0));
      }
      // trailing update A22 <- H^H A22 H
      z64* A22 = A + (k0 + b) + (int64_t)(k0 + b) * lda;
      z64* Yb = V3c + (int64_t)b * ld3;
      gemm_hn<double>(st, m, m, b, A22, lda, V3c, ld3, X, ld3, 1.0, 0.0, part);  // A22^H V = A22 V
      // Y = X T, N = V^H Y, M = T^H N, Z = Y - V M / 2 (over Y), and with
      // look-ahead the next panel's columns of A22 -= V Z^H + Z V^H
      const int nbk = (m + kBw - 1) / kBw;
      const int upd = (look && m > b) ? 1 : 0;
      hipLaunchKernelGGL(k_wy_y, dim3(nbk), dim3(1024), 0, st, m, X, ld3, Tp, V3c, ld3, Yb, ld3, Npart);
      int64_t nfill = 0;
      if (k0 + 2 * b < q) {
        const int m1 = m - b, ns1 = std::min(b, m1), G1 = (m1 + kPanelRows - 1) / kPanelRows;
        nfill = (int64_t)2 * ns1 * (G1 + 1) * 64;
      }
      hipLaunchKernelGGL(k_wy_m, dim3(kBw), dim3(256), 0, st, m, nbk, Npart, Tp, Mm, V3c, ld3, Yb, ld3,
                         reinterpret_cast<unsigned long long*>(slots), nfill);
      hipLaunchKernelGGL(k_wy_z, dim3(nbk), dim3(1024), 0, st, m, Mm, V3c, ld3, Yb, ld3, A22, lda, upd);
      HIPCK(hipGetLastError());
      if (upd) {
        // the rest after the next panel's launch
        HIPCK(hipEventRecord(aux->z, st));
        rest = Deferred{true, true, m, k0, ns, idx, V3c, Yb, A22};
      } else {
        gemm_nn<double>(st, m, 2 * b, m, V3c, ld3, Yb, ld3, 1, A22, lda, -1.0, 0.0, 1.0);
        if (fwd_on_aux) {
          // no deferred update: the forward application of this panel right away
          if (rest.on) submit_rest();
          HIPCK(hipEventRecord(aux->z, st));
          rest = Deferred{true, false, m, k0, ns, idx, V3c, Yb, A22};
          submit_rest();
        }
      }
    }
    if (rest.on) {
      const bool had_upd = rest.upd;
      submit_rest();
      if (had_upd) HIPCK(hipStreamWaitEvent(st, aux->c, 0));
    }
    if (fwd_on_aux) HIPCK(hipStreamWaitEvent(st, aux->f, 0));
    int bad = 0;
    HIPCK(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (bad != 0) fail(EAHP_EDEVICE, "exchange wait of the band reduction timed out");
  }
  hipLaunchKernelGGL(k_band_rows, dim3((unsigned)std::min<int64_t>(8192, ((int64_t)q * kRw + 255) / 256)), dim3(256),
                     0, st, q, A, lda, RB);
  const bool fwd_done = aux != nullptr && aux->s != nullptr && aux->part != nullptr && aux->f != nullptr;
  auto gepp = [&](int lb, int le) {
    for (int l0 = lb; l0 < le; l0 += nsh) {
      const int n = std::min(nsh, le - l0);
      hipLaunchKernelGGL(k_band_gepp, dim3(n), dim3(kGt), 0, st, q, RB, s, Yt, (int64_t)q, Ubuf, l0);
    }
  };
  // Q^H C~ (unless it ran during the reduction, on the second stream), every
  // shift's elimination in one launch where the kept rows allow (one
  // work-group per CU at a time: the shifts beyond the first round start as
  // CUs free up, with no gap between launches), then Q y over all columns.
  if (!fwd_done) apply_refl_blocked(st, q, b, p, Vh, bt, Yt, q, 1, wy, part);
  gepp(0, p);
  apply_refl_blocked(st, q, b, p, Vh, bt, Yt, q, 0, wy, part);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
