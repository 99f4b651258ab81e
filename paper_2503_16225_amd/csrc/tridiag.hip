// Projected Sylvester solve of the block FOM (Algorithm 4): A Y - Y Sigma = C
// with A (q x q) and Sigma (p x p) Hermitian.  In the eigenbasis of
// Sigma = U diag(s) U^H the columns decouple into (A - s_l I) y~_l = c~_l.
// A is reduced once to Hermitian tridiagonal form A = Q T Q^H with Householder
// reflectors (a cooperative kernel over several work-groups, one grid barrier
// per column), after which every shifted system is a tridiagonal solve:
//
//   y~_l = Q (T - s_l I)^-1 Q^H c~_l.
//
// The result is the same Galerkin solution as with a full eigendecomposition
// of A (it is unique), at the cost of one reduction of A per FOM iteration.
// Up to q = 512 the reduction keeps A in registers and its work-groups hand
// each other the data of every step through polled exchange slots; larger q
// use an L2-resident variant with the cooperative groups barrier.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>

#include "devcommon.h"
#include "exchange.h"
#include "kernels.h"
#include "ops.h"

namespace cg = cooperative_groups;

namespace eahp {

using xch::kEmpty;
using xch::poll_z;
using xch::put_z;

// Householder tridiagonalisation.  Column k: x = A[k+1:, k] (length m),
// alpha = -(x0/|x0|) ||x||, v = x - alpha e1, H = I - beta v v^H with
// beta = 2 / v^H v (Hermitian, H x = alpha e1); trailing block
// A' = H A H via p = beta A v, w = p - (beta/2)(v^H p) v, A' = A - v w^H - w v^H.
// Outputs: d (diagonal), e (sub-diagonal T[k+1][k]), the reflectors
// Vh[k+1:, k] and beta[k].  A is destroyed.
//
// Column c of A is owned by work-group c mod G.  One grid barrier per column:
// after it every work-group holds p (global), forms w, updates its own
// columns c >= k+2, and recomputes the updated column k+1 itself (nobody
// writes column k+1 in step k), from which it forms the next reflector and
// the next p entries of its own columns (double-buffered p).
//
// The trailing matrix is stored as TA: complex128, or complex64 for the
// single-precision metric solve (every step still computes in FP64 and rounds
// the updated entries once, on the store).
__device__ __forceinline__ z64 tr_ld(const z64& a) { return a; }
__device__ __forceinline__ z64 tr_ld(const c32& a) { return mk<double>((double)a.x, (double)a.y); }
__device__ __forceinline__ void tr_st(z64* p, z64 a) { *p = a; }
__device__ __forceinline__ void tr_st(c32* p, z64 a) { *p = mk<float>((float)a.x, (float)a.y); }

template <typename TA>
__device__ void tri_reflector(int m, const TA* x_in, z64* v, double* red, double* sc, z64& alpha, double& b) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double s2 = 0;
  for (int i = tid; i < m; i += nt) {
    const z64 t = x_in ? tr_ld(x_in[i]) : v[i];
    v[i] = t;
    s2 += t.x * t.x + t.y * t.y;
  }
  s2 = block_sum(s2, red);
  if (tid == 0) sc[0] = s2;
  __syncthreads();
  const double xn = sqrt(sc[0]);
  const z64 x0 = v[0];
  const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
  if (a0 > 0) alpha = mk<double>(-x0.x / a0 * xn, -x0.y / a0 * xn);
  else alpha = mk<double>(-xn, 0.0);
  const z64 v0 = csub<double>(x0, alpha);
  const double vv = (sc[0] - a0 * a0) + (v0.x * v0.x + v0.y * v0.y);
  b = vv > 0 ? 2.0 / vv : 0.0;
  __syncthreads();
  if (tid == 0) v[0] = v0;
  __syncthreads();
}

// Work items of the trailing columns: column c of A belongs to work-group
// c mod G in every step (so it stays in that work-group's L2), and the
// work-group's waves split its columns into chunks of kTrChunk rows, one
// (column, chunk) item per wave at a time.  Each item leaves the partial sum
// of its rows of an entry of p in slot [chunk][entry]; the readers of p add
// the chunks in chunk order, so p does not depend on G.
constexpr int kTrRB = 8;               // rows per lane of one item
constexpr int kTrChunk = 64 * kTrRB;   // rows of one item
__host__ __device__ constexpr int tr_nch(int m) { return m > 0 ? (m + kTrChunk - 1) / kTrChunk : 1; }

// p of step 0: slot [ch][c - 1] = b * (rows of chunk ch of A[1:, c])^H v, c >= 1
template <typename TA>
__device__ void tri_matvec0(int q, int G, const TA* A, int64_t lda, const z64* v, double b, z64* P) {
  const int m = q - 1, nch = tr_nch(m);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int g = blockIdx.x;
  const int c0 = 1 + ((g - 1) % G + G) % G;
  const int ncolg = c0 < q ? (q - 1 - c0) / G + 1 : 0;
  for (int t = wave; t < ncolg * nch; t += nw) {
    const int c = c0 + (t % ncolg) * G, ch = t / ncolg;
    const TA* col = A + 1 + (int64_t)c * lda;
    const int r0 = ch * kTrChunk + lane;
    z64 a[kTrRB];
#pragma unroll
    for (int u = 0; u < kTrRB; ++u) {
      const int r = r0 + 64 * u;
      a[u] = r < m ? tr_ld(col[r]) : mk<double>(0.0, 0.0);
    }
    double sx = 0, sy = 0;
#pragma unroll
    for (int u = 0; u < kTrRB; ++u) {
      const int r = r0 + 64 * u;
      if (r < m) {
        const z64 vr = v[r];
        sx += a[u].x * vr.x + a[u].y * vr.y;
        sy += a[u].x * vr.y - a[u].y * vr.x;
      }
    }
    sx = warp_sum(sx);
    sy = warp_sum(sy);
    if (lane == 0) P[(int64_t)ch * q + (c - 1)] = mk<double>(b * sx, b * sy);
  }
}

// The work-group's vectors v, w and vn (3 q values) live in LDS, or, when
// vbuf is not null (q too large for LDS), in the work-group's own 3 q slice of
// vbuf in global memory.
template <typename TA>
__global__ void __launch_bounds__(1024) k_tridiag(int q, TA* A, int64_t lda, double* d, z64* e, z64* Vh,
                                                  int64_t ldv, double* beta, z64* Pbuf, z64* vbuf) {
  extern __shared__ unsigned char smem_raw[];
  z64* v = vbuf ? vbuf + (int64_t)3 * q * blockIdx.x : reinterpret_cast<z64*>(smem_raw);  // q
  z64* w = v + q;                             // q
  z64* vn = w + q;                            // q: next reflector
  __shared__ double red[32];
  __shared__ double sc[4];
  cg::grid_group grid = cg::this_grid();
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  // step 0 reflector and p
  z64 alpha;
  double b;
  tri_reflector(q - 1, A + 1, v, red, sc, alpha, b);
  if (g == 0) {
    for (int i = tid; i < q - 1; i += nt) Vh[1 + i] = v[i];
    if (tid == 0) Vh[0] = mk<double>(0.0, 0.0);
    if (tid == 0) {
      d[0] = tr_ld(A[0]).x;
      e[0] = alpha;
      beta[0] = b;
    }
  }
  const int64_t pst = (int64_t)tr_nch(q - 1) * q;  // slots of one buffer of p partials
  tri_matvec0(q, G, A, lda, v, b, Pbuf);
  grid.sync();
  for (int k = 0; k + 1 < q; ++k) {
    const int m = q - k - 1;
    const z64* P = Pbuf + (k & 1) * pst;
    z64* Pn = Pbuf + ((k + 1) & 1) * pst;
    // chunks of the partials of this step's p (written over m + 1 rows in
    // step k - 1, over m rows by tri_matvec0)
    const int nrd = tr_nch(k == 0 ? m : m + 1);
    // w = p - (beta/2)(v^H p) v
    double kx = 0;
    for (int i = tid; i < m; i += nt) {
      // the first 8 chunks loaded together, added in chunk order
      z64 t[8];
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) t[ch] = ch < nrd ? P[(int64_t)ch * q + i] : mk<double>(0.0, 0.0);
      z64 pi = t[0];
#pragma unroll
      for (int ch = 1; ch < 8; ++ch)
        if (ch < nrd) {
          pi.x += t[ch].x;
          pi.y += t[ch].y;
        }
      for (int ch = 8; ch < nrd; ++ch) {
        const z64 u = P[(int64_t)ch * q + i];
        pi.x += u.x;
        pi.y += u.y;
      }
      w[i] = pi;
      kx += v[i].x * pi.x + v[i].y * pi.y;
    }
    kx = block_sum(kx, red);
    if (tid == 0) sc[1] = 0.5 * b * kx;
    __syncthreads();
    const double K = sc[1];
    for (int i = tid; i < m; i += nt) w[i] = mk<double>(w[i].x - K * v[i].x, w[i].y - K * v[i].y);
    __syncthreads();
    if (m == 1) {
      // last step: only the 1 x 1 trailing block remains
      if (g == 0 && tid == 0) {
        const z64 a = tr_ld(A[(k + 1) + (int64_t)(k + 1) * lda]);
        const double u = 2.0 * (v[0].x * w[0].x + v[0].y * w[0].y);
        d[k + 1] = a.x - u;
      }
      break;
    }
    // updated column k+1 (rows k+2..), recomputed redundantly (nobody writes
    // column k+1 in step k): x = A[k+2:, k+1] - v w_0^* - w v_0^*
    const int m2 = m - 1;
    {
      const TA* colk1 = A + (k + 2) + (int64_t)(k + 1) * lda;
      const z64 w0 = w[0], v0 = v[0];
      for (int r = tid; r < m2; r += nt) {
        const z64 vr = v[r + 1], wr = w[r + 1];
        const double ux = vr.x * w0.x + vr.y * w0.y + wr.x * v0.x + wr.y * v0.y;
        const double uy = vr.y * w0.x - vr.x * w0.y + wr.y * v0.x - wr.x * v0.y;
        const z64 a = tr_ld(colk1[r]);
        vn[r] = mk<double>(a.x - ux, a.y - uy);
      }
    }
    double dk1 = 0;
    if (tid == 0) {
      const z64 a = tr_ld(A[(k + 1) + (int64_t)(k + 1) * lda]);
      dk1 = a.x - 2.0 * (v[0].x * w[0].x + v[0].y * w[0].y);
    }
    __syncthreads();
    // next reflector from vn (in place), before the trailing update
    z64 an;
    double bn;
    tri_reflector<TA>(m2, nullptr, vn, red, sc, an, bn);
    if (g == 0) {
      for (int i = tid; i < m2; i += nt) Vh[(k + 2 + i) + (int64_t)(k + 1) * ldv] = vn[i];
      for (int i = tid; i < k + 2; i += nt) Vh[i + (int64_t)(k + 1) * ldv] = mk<double>(0.0, 0.0);
      if (tid == 0) {
        d[k + 1] = dk1;
        e[k + 1] = an;
        beta[k + 1] = bn;
      }
    }
    // one pass over every owned item (column c >= k + 2, chunk of rows): the
    // rank-2 update A -= v w^H + w v^H, stored back, and in the same pass
    // the chunk's part of the entry of p of step k+1, bn (A[k+2:, c])^H vn
    {
      const int cf = k + 2;
      const int c0 = cf + ((g - cf) % G + G) % G;
      const int ncolg = c0 < q ? (q - 1 - c0) / G + 1 : 0;
      const int nch = tr_nch(m);
      for (int t = wave; t < ncolg * nch; t += nw) {
        const int c = c0 + (t % ncolg) * G, ch = t / ncolg;
        const int j = c - (k + 1);
        const z64 wj = w[j], vj = v[j];
        TA* col = A + (k + 1) + (int64_t)c * lda;
        const int r0 = ch * kTrChunk + lane;
        // the item's loads are issued together, so their latency is paid once
        z64 a0[kTrRB];
#pragma unroll
        for (int u = 0; u < kTrRB; ++u) {
          const int r = r0 + 64 * u;
          a0[u] = r < m ? tr_ld(col[r]) : mk<double>(0.0, 0.0);
        }
        double sx = 0, sy = 0;
#pragma unroll
        for (int u = 0; u < kTrRB; ++u) {
          const int r = r0 + 64 * u;
          if (r < m) {
            const z64 vr = v[r], wr = w[r];
            const double ux = vr.x * wj.x + vr.y * wj.y + wr.x * vj.x + wr.y * vj.y;
            const double uy = vr.y * wj.x - vr.x * wj.y + wr.y * vj.x - wr.x * vj.y;
            const z64 a = mk<double>(a0[u].x - ux, a0[u].y - uy);
            tr_st(col + r, a);
            if (r >= 1) {
              const z64 x = vn[r - 1];
              sx += a.x * x.x + a.y * x.y;
              sy += a.x * x.y - a.y * x.x;
            }
          }
        }
        sx = warp_sum(sx);
        sy = warp_sum(sy);
        if (lane == 0) Pn[(int64_t)ch * q + (c - (k + 2))] = mk<double>(bn * sx, bn * sy);
      }
    }
    __syncthreads();
    for (int i = tid; i < m2; i += nt) v[i] = vn[i];
    b = bn;
    __syncthreads();
    grid.sync();
  }
}

// ---------------------------------------------------------------------------
// Register-resident reduction for q <= 64 NS.  Every wave holds two whole
// columns of A (row i in lane i % 64, slot i / 64) and its own copy of the
// reflector v, of w and of the next column, so every inner product is a
// wave reduction and the only exchange between waves is the vector p of each
// step: its entries (one per owned column) and the next column to be reduced
// go to global memory, followed by one grid barrier (a counter in global
// memory; the waits are bounded and a timeout is reported through *err).
namespace {
constexpr int kTrWaves = 8;  // waves per work-group
constexpr int kTrCols = 2;   // columns per wave

// Row r (wave-uniform) of a register-distributed vector, in every lane.  The
// lane read happens inside the branch of the matching slot, so that no slot
// is selected by a computed index (which would move the array to scratch).
template <int NS> __device__ __forceinline__ z64 pick_row(const z64 (&x)[NS], int r) {
  z64 t = mk<double>(0.0, 0.0);
  const int sl = r >> 6, l = r & 63;
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (sl == s) t = mk<double>(readlane_f64(x[s].x, l), readlane_f64(x[s].y, l));
  return t;
}

// Householder vector from x (rows >= r0, zero elsewhere): x[r0] -= alpha.
template <int NS> __device__ __forceinline__ void reflector_reg(z64 (&x)[NS], int r0, z64& alpha, double& b) {
  double s2 = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) s2 += x[s].x * x[s].x + x[s].y * x[s].y;
  s2 = wave_allsum(s2);
  const z64 x0 = pick_row<NS>(x, r0);
  const double xn = sqrt(s2);
  const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
  if (a0 > 0) alpha = mk<double>(-x0.x / a0 * xn, -x0.y / a0 * xn);
  else alpha = mk<double>(-xn, 0.0);
  const z64 v0 = csub<double>(x0, alpha);
  const double vv = (s2 - a0 * a0) + (v0.x * v0.x + v0.y * v0.y);
  b = vv > 0 ? 2.0 / vv : 0.0;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (lane + 64 * s == r0) x[s] = v0;
}

}  // namespace

template <int NS>
__global__ void __launch_bounds__(64 * kTrWaves) k_tridiag_reg(int q, const z64* __restrict__ A, int64_t lda,
                                                               int64_t sA, double* d, z64* e, z64* Vh, int64_t ldv,
                                                               int64_t sV, double* beta, z64* Pb, z64* Cb,
                                                               int64_t sx, int* err) {
  // Pb, Cb: q x q exchange slots (row k = step k) holding the kEmpty pattern.
  // blockIdx.y: the matrix of a batch (A, Vh and the slots at strides sA, sV,
  // sx; d, e and beta at stride q); the work-groups of one matrix exchange
  // only among themselves
  A += blockIdx.y * sA;
  Vh += blockIdx.y * sV;
  Pb += blockIdx.y * sx;
  Cb += blockIdx.y * sx;
  d += (int64_t)blockIdx.y * q;
  e += (int64_t)blockIdx.y * q;
  beta += (int64_t)blockIdx.y * q;
  __shared__ z64 sP[2][64 * NS], sC[2][64 * NS];
  __shared__ int sbad;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int G = gridDim.x;
  const int nwt = G * kTrWaves;
  const int gw = blockIdx.x * kTrWaves + wv;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  int col[kTrCols];
  z64 a[kTrCols][NS];
#pragma unroll
  for (int j = 0; j < kTrCols; ++j) {
    col[j] = gw + j * nwt;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      a[j][s] = (col[j] < q && i < q) ? A[i + (int64_t)col[j] * lda] : mk<double>(0.0, 0.0);
    }
  }
  // reflector 0 from column 0 (rows 1..q-1)
  z64 v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    v[s] = (i >= 1 && i < q) ? A[i] : mk<double>(0.0, 0.0);
  }
  z64 alpha;
  double b;
  reflector_reg<NS>(v, 1, alpha, b);
  if (gw == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (lane + 64 * s < q) Vh[lane + 64 * s] = v[s];
    if (lane == 0) {
      d[0] = A[0].x;
      e[0] = alpha;
      beta[0] = b;
    }
  }
  // p_0 entries of the owned columns c >= 1
#pragma unroll
  for (int j = 0; j < kTrCols; ++j) {
    if (col[j] >= 1 && col[j] < q) {
      double sx = 0, sy = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        sx += a[j][s].x * v[s].x + a[j][s].y * v[s].y;
        sy += a[j][s].x * v[s].y - a[j][s].y * v[s].x;
      }
      sx = wave_allsum(sx);
      sy = wave_allsum(sy);
      if (lane == 0) put_z(Pb + col[j], mk<double>(b * sx, b * sy));
    }
  }
  for (int k = 0; k + 1 < q; ++k) {
    // p_k and the column k+1 as updated through step k-1 (rows k+1..), polled
    // by the threads of the work-group into LDS (double-buffered by step)
    {
      const int t = threadIdx.x;
      if (t >= k + 1 && t < q) {
        bool ok = true;
        sP[k & 1][t] = poll_z(Pb + (int64_t)k * q + t, ok);
        sC[k & 1][t] = k == 0 ? A[t + lda] : poll_z(Cb + (int64_t)k * q + t, ok);
        if (!ok) sbad = 1;
      }
      __syncthreads();
      if (sbad) {
        if (threadIdx.x == 0) *reinterpret_cast<volatile int*>(err) = 1;
        return;
      }
    }
    // w = p - (beta/2)(v^H p) v
    z64 w[NS], cc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      const bool in = i >= k + 1 && i < q;
      w[s] = in ? sP[k & 1][i] : mk<double>(0.0, 0.0);
      cc[s] = in ? sC[k & 1][i] : mk<double>(0.0, 0.0);
    }
    double kx = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) kx += v[s].x * w[s].x + v[s].y * w[s].y;
    const double K = 0.5 * b * wave_allsum(kx);
#pragma unroll
    for (int s = 0; s < NS; ++s) w[s] = mk<double>(w[s].x - K * v[s].x, w[s].y - K * v[s].y);
    const z64 v1 = pick_row<NS>(v, k + 1), w1 = pick_row<NS>(w, k + 1), c1 = pick_row<NS>(cc, k + 1);
    const double dk1 = c1.x - 2.0 * (v1.x * w1.x + v1.y * w1.y);
    if (k + 2 == q) {
      if (gw == 0 && lane == 0) d[k + 1] = dk1;
      break;
    }
    // next reflector from x = A'[k+2:, k+1] = c - v conj(w1) - w conj(v1)
    z64 x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      if (i >= k + 2) {
        const double ux = v[s].x * w1.x + v[s].y * w1.y + w[s].x * v1.x + w[s].y * v1.y;
        const double uy = v[s].y * w1.x - v[s].x * w1.y + w[s].y * v1.x - w[s].x * v1.y;
        x[s] = mk<double>(cc[s].x - ux, cc[s].y - uy);
      } else {
        x[s] = mk<double>(0.0, 0.0);
      }
    }
    z64 an;
    double bn;
    reflector_reg<NS>(x, k + 2, an, bn);
    // rank-2 update of the owned columns c >= k+2 and their entries of p_{k+1}
    z64* Pn = Pb + (int64_t)(k + 1) * q;
#pragma unroll
    for (int j = 0; j < kTrCols; ++j) {
      const int c = col[j];
      if (c >= k + 2 && c < q) {
        const z64 vc = pick_row<NS>(v, c), wc = pick_row<NS>(w, c);
        double sx = 0, sy = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const double ux = v[s].x * wc.x + v[s].y * wc.y + w[s].x * vc.x + w[s].y * vc.y;
          const double uy = v[s].y * wc.x - v[s].x * wc.y + w[s].y * vc.x - w[s].x * vc.y;
          a[j][s] = mk<double>(a[j][s].x - ux, a[j][s].y - uy);
          sx += a[j][s].x * x[s].x + a[j][s].y * x[s].y;
          sy += a[j][s].x * x[s].y - a[j][s].y * x[s].x;
        }
        sx = wave_allsum(sx);
        sy = wave_allsum(sy);
        if (lane == 0) put_z(Pn + c, mk<double>(bn * sx, bn * sy));
        if (c == k + 2) {
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int i = lane + 64 * s;
            if (i >= k + 2 && i < q) put_z(Cb + (int64_t)(k + 1) * q + i, a[j][s]);
          }
        }
      }
    }
    if (gw == 0) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (lane + 64 * s < q) Vh[lane + 64 * s + (int64_t)(k + 1) * ldv] = x[s];
      if (lane == 0) {
        d[k + 1] = dk1;
        e[k + 1] = an;
        beta[k + 1] = bn;
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = x[s];
    b = bn;
  }
}

// H_k b = b - beta_k v_k (v_k^H b) for k = 0..q-2 (forward: Q^H B) or
// k = q-2..0 (backward: Q B), one wave per column of B held in registers;
// the reflector of the next step is loaded while the current one is applied.
template <int NS>
__global__ void __launch_bounds__(256) k_apply_refl_reg(int q, const z64* __restrict__ Vh, int64_t ldv,
                                                        const double* __restrict__ beta, z64* B, int64_t ldb,
                                                        int ncols, int forward, int64_t sV, int64_t sB) {
  // blockIdx.y: the matrix of a batch (Vh, B at strides sV, sB; beta at q)
  Vh += blockIdx.y * sV;
  B += blockIdx.y * sB;
  beta += (int64_t)blockIdx.y * q;
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (l >= ncols || q < 2) return;
  z64* bc = B + (int64_t)l * ldb;
  z64 x[NS], vn[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    x[s] = i < q ? bc[i] : mk<double>(0.0, 0.0);
  }
  const int nr = q - 1;
  auto load = [&](int k) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + 64 * s;
      vn[s] = (i > k && i < q) ? Vh[i + (int64_t)k * ldv] : mk<double>(0.0, 0.0);
    }
  };
  load(forward ? 0 : nr - 1);
  for (int t = 0; t < nr; ++t) {
    const int k = forward ? t : nr - 1 - t;
    z64 v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = vn[s];
    if (t + 1 < nr) load(forward ? k + 1 : k - 1);
    double sx = 0, sy = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      sx += v[s].x * x[s].x + v[s].y * x[s].y;
      sy += v[s].x * x[s].y - v[s].y * x[s].x;
    }
    const double bk = beta[k];
    const z64 f = mk<double>(bk * wave_allsum(sx), bk * wave_allsum(sy));
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = csub<double>(x[s], cmul<double>(v[s], f));
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lane + 64 * s;
    if (i < q) bc[i] = x[s];
  }
}

// (T - s_l I) y = b for every column l, Gaussian elimination with partial
// pivoting between adjacent rows, one thread per column.  The running row and
// right-hand side stay in registers; the finished rows (inverse of the pivot,
// first and second super-diagonal) go to W with the columns interleaved
// (coalesced).
__global__ void __launch_bounds__(64) k_trisolve_reg(int q, int ncols, const double* __restrict__ d,
                                                     const z64* __restrict__ e, const double* __restrict__ sh,
                                                     z64* B, int64_t ldb, z64* W, int64_t sB) {
  // blockIdx.y: the system of a batch (d, e at stride q, the shifts at
  // ncols, B at sB, W at 3 q ncols)
  d += (int64_t)blockIdx.y * q;
  e += (int64_t)blockIdx.y * q;
  sh += (int64_t)blockIdx.y * ncols;
  B += blockIdx.y * sB;
  W += (int64_t)blockIdx.y * 3 * q * ncols;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ncols) return;
  z64* b = B + (int64_t)l * ldb;
  auto row = [&](int i, int c) -> z64& { return W[((int64_t)3 * i + c) * ncols + l]; };
  // 1/c = conj(c) / |c|^2
  auto rinv = [](z64 c) {
    const double r = 1.0 / (c.x * c.x + c.y * c.y);
    return mk<double>(c.x * r, -c.y * r);
  };
  const double s = sh[l];
  z64 Dc = mk<double>(d[0] - s, 0.0);
  z64 Uc = q > 1 ? mk<double>(e[0].x, -e[0].y) : mk<double>(0.0, 0.0);
  z64 bc = b[0];
  // forward elimination with row pivoting (the larger of |Dc|, |L| as the
  // pivot, compared squared); each row keeps the inverse of its pivot, so
  // the back substitution has no division on its dependency chain.  The
  // entries of a block of rows are loaded together before the block is
  // eliminated, one memory latency per block instead of per row.
  constexpr int PB = 16;
  for (int i0 = 0; i0 + 1 < q; i0 += PB) {
    z64 Lb[PB], Ub[PB], Bb[PB];
    double Db[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) {
      const int i = i0 + j;
      if (i + 1 < q) {
        Lb[j] = e[i];
        Db[j] = d[i + 1];
        Ub[j] = i + 2 < q ? mk<double>(e[i + 1].x, -e[i + 1].y) : mk<double>(0.0, 0.0);
        Bb[j] = b[i + 1];
      }
    }
#pragma unroll
    for (int j = 0; j < PB; ++j) {
      const int i = i0 + j;
      if (i + 1 < q) {
        const z64 L = Lb[j];
        const z64 Dn = mk<double>(Db[j] - s, 0.0);
        const z64 Un = Ub[j];
        const z64 bn = Bb[j];
        if (Dc.x * Dc.x + Dc.y * Dc.y >= L.x * L.x + L.y * L.y) {
          const z64 iD = rinv(Dc);
          const z64 f = cmul<double>(L, iD);
          row(i, 0) = iD;
          row(i, 1) = Uc;
          row(i, 2) = mk<double>(0.0, 0.0);
          b[i] = bc;
          Dc = csub<double>(Dn, cmul<double>(f, Uc));
          Uc = Un;
          bc = csub<double>(bn, cmul<double>(f, bc));
        } else {
          const z64 iL = rinv(L);
          const z64 f = cmul<double>(Dc, iL);
          row(i, 0) = iL;
          row(i, 1) = Dn;
          row(i, 2) = Un;
          b[i] = bn;
          const z64 Dnew = csub<double>(Uc, cmul<double>(f, Dn));
          Uc = mk<double>(-(f.x * Un.x - f.y * Un.y), -(f.x * Un.y + f.y * Un.x));
          bc = csub<double>(bc, cmul<double>(f, bn));
          Dc = Dnew;
        }
      }
    }
  }
  // back substitution, x_{i+1} and x_{i+2} carried in registers, blocks of
  // rows loaded ahead as above
  z64 x1 = cmul<double>(bc, rinv(Dc)), x2 = mk<double>(0.0, 0.0);
  b[q - 1] = x1;
  for (int i1 = q - 2; i1 >= 0; i1 -= PB) {
    z64 R0[PB], R1[PB], R2[PB], Bb[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) {
      const int i = i1 - j;
      if (i >= 0) {
        R0[j] = row(i, 0);
        R1[j] = row(i, 1);
        R2[j] = row(i, 2);
        Bb[j] = b[i];
      }
    }
#pragma unroll
    for (int j = 0; j < PB; ++j) {
      const int i = i1 - j;
      if (i >= 0) {
        z64 r = csub<double>(Bb[j], cmul<double>(R1[j], x1));
        r = csub<double>(r, cmul<double>(R2[j], x2));
        const z64 xi = cmul<double>(r, R0[j]);
        b[i] = xi;
        x2 = x1;
        x1 = xi;
      }
    }
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Apply the reflectors to the columns of B (q x ncols, ld ldb), one work-group
// per column: forward (Q^H B = H_{q-2} ... H_0 B) or backward (Q B).
__global__ void __launch_bounds__(256) k_apply_refl(int q, const z64* Vh, int64_t ldv, const double* beta, z64* B,
                                                    int64_t ldb, int forward) {
  __shared__ double red[32];
  __shared__ z64 dotv;
  z64* bc = B + (int64_t)blockIdx.x * ldb;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int s = 0; s + 1 < q; ++s) {
    const int k = forward ? s : q - 2 - s;
    const int m = q - k - 1;
    const z64* v = Vh + (k + 1) + (int64_t)k * ldv;
    z64* bb = bc + k + 1;
    double sx = 0, sy = 0;
    for (int r = tid; r < m; r += nt) {
      const z64 a = v[r], x = bb[r];
      sx += a.x * x.x + a.y * x.y;
      sy += a.x * x.y - a.y * x.x;
    }
    sx = block_sum(sx, red);
    sy = block_sum(sy, red + 16);
    if (tid == 0) dotv = mk<double>(beta[k] * sx, beta[k] * sy);
    __syncthreads();
    const z64 f = dotv;
    for (int r = tid; r < m; r += nt) bb[r] = csub<double>(bb[r], cmul<double>(v[r], f));
    __syncthreads();
  }
}

__device__ __forceinline__ double cabs_(z64 a) { return sqrt(a.x * a.x + a.y * a.y); }
__device__ __forceinline__ z64 cdiv_(z64 a, z64 b) {
  const double den = b.x * b.x + b.y * b.y;
  return mk<double>((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__global__ void k_set_d0(const z64* A, double* d) { d[0] = A[0].x; }

namespace {
template <int NS>
void tridiag_reg_launch(hipStream_t st, int q, const z64* A, int64_t lda, double* dd, z64* e, z64* Vh, double* bt,
                        z64* Pb, z64* Cb, int* herr) {
  const int G = (q + kTrWaves * kTrCols - 1) / (kTrWaves * kTrCols);
  // Pb and Cb are contiguous: 2 q^2 complex slots, 4 q^2 words; the error
  // flag (device memory) follows them and starts at zero
  const int64_t nw = (int64_t)4 * q * q;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>(1024, (nw + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(Pb), nw, kEmpty);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned long long*>(herr), (int64_t)1,
                     0ull);
  int qq = q;
  int64_t la = lda, lv = q;
  int64_t s0 = 0;
  void* args[] = {&qq, &A, &la, &s0, &dd, &e, &Vh, &lv, &s0, &bt, &Pb, &Cb, &s0, &herr};
  HIPCK(hipLaunchCooperativeKernel((const void*)k_tridiag_reg<NS>, dim3(G), dim3(64 * kTrWaves), args, 0, st));
  int bad = 0;
  HIPCK(hipMemcpyAsync(&bad, herr, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  if (bad != 0) fail(EAHP_EDEVICE, "exchange wait of the tridiagonal reduction timed out");
}

// Work-groups of the L2-resident reduction; its vectors stay in LDS up to
// q = kTrLdsMax (3 q complex values per work-group).
constexpr int kTrLdsMax = 3200;
// columns per work-group of the candidates of the autotuner (candidate 0:
// one work-group per 32 columns, the default)
constexpr int kTrCpw[] = {32, 16, 8, 64};
constexpr int kTrNcand = 4;
int tridiag_groups(int q, int cpw = 32) {
  int dev = 0, ncu = 0;
  HIPCK(hipGetDevice(&dev));
  HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  return std::min(ncu, std::max(1, (q + cpw - 1) / cpw));
}
}  // namespace

// Kernels that wait on each other's work-groups must not share the CUs with
// another such launch from a concurrent stream (the serving loop): one at a
// time per process, waited for before the next.
std::mutex& coop_mutex() {
  static std::mutex m;
  return m;
}

size_t tridiag_scratch(int q) {
  if (q < 2) return 0;
  if (q <= 512) return sizeof(z64) * 2 * (size_t)q * q + 64;  // exchange slots, error flag
  size_t b = sizeof(z64) * 2 * (size_t)tr_nch(q - 1) * q;  // double-buffered partials of p
  int gmax = 1;
  for (int c = 0; c < kTrNcand; ++c) gmax = std::max(gmax, tridiag_groups(q, kTrCpw[c]));
  if (q > kTrLdsMax) b += sizeof(z64) * 3 * (size_t)q * gmax;
  return b;
}

namespace {
// the multi-work-group reduction (q > 512); the caller holds coop_mutex()
template <typename TA>
void tridiag_l2(hipStream_t st, int q, TA* A, int64_t lda, double* dd, z64* e, z64* Vh, double* bt, void* scr) {
  const bool gvec = q > kTrLdsMax;
  z64* P = static_cast<z64*>(scr);
  z64* vb = gvec ? P + 2 * (size_t)tr_nch(q - 1) * q : nullptr;
  const size_t lds = gvec ? 0 : sizeof(z64) * 3 * (size_t)q;
  const void* kern = (const void*)k_tridiag<TA>;
  HIPCK(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 1024, lds));
  if (per_cu < 1) fail(EAHP_EDEVICE, "the tridiagonal reduction cannot be made resident");
  // work-groups: the autotuner's choice for this size class, timed on a copy
  // of A (the results do not depend on it: the row chunks of the columns and
  // the order in which their partial sums are added are the same for every
  // grid, and every work-group forms the same reflectors)
  const int qb = (q + 511) / 512 * 512;
  const std::string key = std::string(sizeof(TA) == 16 ? "k_tridiag<c128>" : "k_tridiag<c64>") + " q<=" +
                          std::to_string(qb);
  const int cand = autotune(st, key, kTrNcand, [&](int c) {
    DevMem Ac, Vc, oc;
    Ac.alloc(sizeof(TA) * (size_t)q * q);
    Vc.alloc(sizeof(z64) * (size_t)q * q);
    oc.alloc(sizeof(z64) * (3 + 2 * (size_t)tr_nch(q - 1)) * q +
             sizeof(z64) * 3 * (size_t)q * tridiag_groups(q, kTrCpw[c]) + 256);
    HIPCK(hipMemcpy2DAsync(Ac.p, sizeof(TA) * q, A, sizeof(TA) * lda, sizeof(TA) * q, q, hipMemcpyDeviceToDevice,
                           st));
    z64* o = oc.as<z64>();
    double* d2 = reinterpret_cast<double*>(o);
    z64* e2 = o + q;
    double* b2 = reinterpret_cast<double*>(o + 2 * q);
    z64* P2 = o + 3 * q;
    z64* vb2 = gvec ? P2 + 2 * (size_t)tr_nch(q - 1) * q : nullptr;
    int qq = q;
    int64_t la = q, lv = q;
    TA* Ap = Ac.as<TA>();
    z64* Vp = Vc.as<z64>();
    void* args[] = {&qq, &Ap, &la, &d2, &e2, &Vp, &lv, &b2, &P2, &vb2};
    HIPCK(hipLaunchCooperativeKernel(kern, dim3(tridiag_groups(q, kTrCpw[c])), dim3(1024), args, lds, st));
    HIPCK(hipStreamSynchronize(st));  // before the temporaries are freed
  });
  const int Gl = tridiag_groups(q, kTrCpw[cand]);
  int qq = q;
  int64_t la = lda, lv = q;
  void* args[] = {&qq, &A, &la, &dd, &e, &Vh, &lv, &bt, &P, &vb};
  // algorithmic bytes: every step reads and writes the live trailing columns
  // (rows k+1.., columns k+2..) once
  double bytes = 0;
  for (int64_t k = 0; k + 2 < q; ++k) bytes += 2.0 * sizeof(TA) * (double)(q - k - 1) * (double)(q - k - 2);
  gemm_prof_begin(st, kProfTridiag);
  HIPCK(hipLaunchCooperativeKernel(kern, dim3(Gl), dim3(1024), args, lds, st));
  gemm_prof_end(st, kProfTridiag, bytes);
  HIPCK(hipStreamSynchronize(st));
}
}  // namespace

void tridiag_reduce(hipStream_t st, int q, z64* A, int64_t lda, double* dd, z64* e, z64* Vh, double* bt, void* scr) {
  if (q <= 0) return;
  if (q == 1) {
    hipLaunchKernelGGL(k_set_d0, dim3(1), dim3(1), 0, st, A, dd);
    HIPCK(hipGetLastError());
    return;
  }
  std::lock_guard<std::mutex> lk(coop_mutex());
  if (q <= 512) {
    z64* Pb = static_cast<z64*>(scr);
    z64* Cb = Pb + (size_t)q * q;
    int* herr = reinterpret_cast<int*>(Cb + (size_t)q * q);
    if (q <= 128) tridiag_reg_launch<2>(st, q, A, lda, dd, e, Vh, bt, Pb, Cb, herr);
    else if (q <= 256) tridiag_reg_launch<4>(st, q, A, lda, dd, e, Vh, bt, Pb, Cb, herr);
    else tridiag_reg_launch<8>(st, q, A, lda, dd, e, Vh, bt, Pb, Cb, herr);
    return;
  }
  tridiag_l2<z64>(st, q, A, lda, dd, e, Vh, bt, scr);
}

void tridiag_reduce(hipStream_t st, int q, c32* A, int64_t lda, double* dd, z64* e, z64* Vh, double* bt, void* scr) {
  if (q <= 512) fail(EAHP_EINVAL, "single-precision storage is for the reduction beyond q = 512");
  std::lock_guard<std::mutex> lk(coop_mutex());
  tridiag_l2<c32>(st, q, A, lda, dd, e, Vh, bt, scr);
}

// Blocks of nb consecutive reflectors P = H_k0 ... H_k0+nb-1 = I - V T V^H
// (compact WY form).  T is not formed: T^-1 = diag(1/beta) + (the strictly
// upper part of G = V^H V), so T Z and T^H Z are triangular solves with G.
// k_wy_trsm solves, for every column z of Z (nbk x ncols, ld ldz) in place,
// (diag(1/beta) + strictly lower G) z2 = z (forward: the factor T^H of P^H)
// or (diag(1/beta) + strictly upper G) z2 = z (backward: T of P); one wave
// per column, entry j in lane j % 64, slot j / 64 (nbk <= 256).
__global__ void __launch_bounds__(256) k_wy_trsm(int nbk, int nb, const z64* __restrict__ G,
                                                 const double* __restrict__ beta, z64* Z, int64_t ldz, int ncols,
                                                 int forward, int64_t sG, int64_t sB, int64_t sZ) {
  // blockIdx.y: the block of reflectors (G, beta and Z at strides sG, sB, sZ)
  G += blockIdx.y * sG;
  beta += blockIdx.y * sB;
  Z += blockIdx.y * sZ;
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (col >= ncols) return;
  z64* zc = Z + (int64_t)col * ldz;
  z64 z[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = lane + 64 * u;
    z[u] = j < nbk ? zc[j] : mk<double>(0.0, 0.0);
  }
  for (int t = 0; t < nbk; ++t) {
    const int i = forward ? t : nbk - 1 - t;
    // column i of G (the entries the other unknowns need)
    z64 gc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = lane + 64 * u;
      gc[u] = j < nbk ? G[j + (int64_t)i * nb] : mk<double>(0.0, 0.0);
    }
    z64 zi = pick_row<4>(z, i);
    const double bi = beta[i];
    zi = mk<double>(bi * zi.x, bi * zi.y);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = lane + 64 * u;
      if (j == i) z[u] = zi;
      else if (forward ? j > i : j < i) z[u] = csub<double>(z[u], cmul<double>(gc[u], zi));
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = lane + 64 * u;
    if (j < nbk) zc[j] = z[u];
  }
}

// identity in the leading n x n of each nb x nb block (blockIdx.y), zero elsewhere
__global__ void k_eye_blocks(int n, int nb, z64* X) {
  X += (int64_t)blockIdx.y * nb * nb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb * nb; e += gridDim.x * blockDim.x) {
    const int i = e % nb, j = e / nb;
    X[e] = mk<double>((i == j && i < n) ? 1.0 : 0.0, 0.0);
  }
}

constexpr int kWyNb = 256;
size_t refl_blocked_scratch(int nref, int ncols) {
  const int nblk = (nref + kWyNb - 1) / kWyNb;
  return sizeof(z64) * (2 * (size_t)nblk * kWyNb * kWyNb + 2 * (size_t)kWyNb * ncols) + 512;
}

// Y <- Q^H Y or Q Y for Q = H_0 H_1 ... H_{nref-1}, reflector k acting on rows
// k + off .. q - 1 (off = 1: the tridiagonal reduction; off = the bandwidth:
// the band reduction), through blocks of kWyNb reflectors P = I - V T V^H.
// T^H = (diag(1/beta) + strictly lower G)^-1 (G = V^H V) of every block is
// formed first, all blocks in one launch (k_wy_trsm on identity right-hand
// sides); per block then three products: Z = V^H Y, T^H Z (forward: the
// factor of P^H) or T Z, Y -= V (T^H Z or T Z).  Column k of Vh must be zero
// above row k + off.
// G and T^H of every block into scr (its first 2 nblk nb^2 values)
void refl_blocked_prepare(hipStream_t st, int q, int off, const z64* Vh, const double* beta, void* scr, DevMem& part) {
  const int nref = q - off;
  if (nref <= 0) return;
  const int nb = kWyNb, nblk = (nref + nb - 1) / nb;
  z64* G = static_cast<z64*>(scr);
  z64* Xi = G + (size_t)nblk * nb * nb;  // T^H of every block
  // G_b = V_b^H V_b: the full blocks at once, then the narrower last one
  const int nfull = nref / nb, last = nref - nfull * nb;
  if (nfull > 0)
    gemm_hn<double>(st, q, nb, nb, Vh, q, Vh, q, G, nb, 1.0, 0.0, part, nfull, (int64_t)nb * q, (int64_t)nb * q,
                    (int64_t)nb * nb);
  if (last > 0)
    gemm_hn<double>(st, q, last, last, Vh + (int64_t)nfull * nb * q, q, Vh + (int64_t)nfull * nb * q, q,
                    G + (int64_t)nfull * nb * nb, nb, 1.0, 0.0, part);
  // T^H of every block: (diag(1/beta) + strictly lower G) X = I
  const int64_t bb = (int64_t)nb * nb;
  if (nfull > 0) {
    hipLaunchKernelGGL(k_eye_blocks, dim3(64, nfull), dim3(256), 0, st, nb, nb, Xi);
    hipLaunchKernelGGL(k_wy_trsm, dim3((nb + 3) / 4, nfull), dim3(256), 0, st, nb, nb, G, beta, Xi, (int64_t)nb, nb,
                       1, bb, (int64_t)nb, bb);
  }
  if (last > 0) {
    z64* Xl = Xi + (int64_t)nfull * bb;
    hipLaunchKernelGGL(k_eye_blocks, dim3(64, 1), dim3(256), 0, st, last, nb, Xl);
    hipLaunchKernelGGL(k_wy_trsm, dim3((last + 3) / 4, 1), dim3(256), 0, st, last, nb, G + (int64_t)nfull * bb,
                       beta + (int64_t)nfull * nb, Xl, (int64_t)nb, last, 1, (int64_t)0, (int64_t)0, (int64_t)0);
  }
  HIPCK(hipGetLastError());
}

// The products with the prepared blocks on ncols columns of Y; zs holds Z
// and Z2 (nb x ncols each).
void refl_blocked_apply(hipStream_t st, int q, int off, int ncols, const z64* Vh, z64* Y, int64_t ldy, int forward,
                        const void* scr, z64* zs, DevMem& part) {
  const int nref = q - off;
  if (nref <= 0 || ncols <= 0) return;
  const int nb = kWyNb, nblk = (nref + nb - 1) / nb;
  const z64* Xi = static_cast<const z64*>(scr) + (size_t)nblk * nb * nb;
  const int64_t bb = (int64_t)nb * nb;
  z64* Z = zs;
  z64* Z2 = Z + (size_t)nb * ncols;
  for (int i = 0; i < nblk; ++i) {
    const int blk = forward ? i : nblk - 1 - i;
    const int k0 = blk * nb, nbk = std::min(nb, nref - k0);
    const int r0 = k0 + off, rows = q - r0;  // the block's reflectors vanish above row k0 + off
    const z64* Vb = Vh + (int64_t)k0 * q + r0;
    const z64* Xb = Xi + (int64_t)blk * bb;
    // Z = V_b^H Y, Z2 = T^H Z (forward) or T Z, Y -= V_b Z2
    gemm_hn<double>(st, rows, nbk, ncols, Vb, q, Y + r0, ldy, Z, nbk, 1.0, 0.0, part);
    if (forward) gemm_nn<double>(st, nbk, nbk, ncols, Xb, nb, Z, nbk, 0, Z2, nbk, 1.0, 0.0, 0.0);
    else gemm_hn<double>(st, nbk, nbk, ncols, Xb, nb, Z, nbk, Z2, nbk, 1.0, 0.0, part);
    gemm_nn<double>(st, rows, nbk, ncols, Vb, q, Z2, nbk, 0, Y + r0, ldy, -1.0, 0.0, 1.0);
  }
  HIPCK(hipGetLastError());
}

void apply_refl_blocked(hipStream_t st, int q, int off, int ncols, const z64* Vh, const double* beta, z64* Y,
                        int64_t ldy, int forward, void* scr, DevMem& part) {
  const int nref = q - off;
  if (nref <= 0 || ncols <= 0) return;
  const int nblk = (nref + kWyNb - 1) / kWyNb;
  refl_blocked_prepare(st, q, off, Vh, beta, scr, part);
  refl_blocked_apply(st, q, off, ncols, Vh, Y, ldy, forward, scr,
                     static_cast<z64*>(scr) + 2 * (size_t)nblk * kWyNb * kWyNb, part);
}

// Q^H Y (forward) or Q Y: a wave per column with the column in registers up to
// q = 512, blocked (compact WY) products beyond
void apply_refl(hipStream_t st, int q, int ncols, const z64* Vh, const double* bt, z64* Y, int64_t ldy, int forward,
                void* wy_scr, DevMem* part) {
  if (q < 2 || ncols <= 0) return;
  if (q > 512 && wy_scr && part) {
    apply_refl_blocked(st, q, 1, ncols, Vh, bt, Y, ldy, forward, wy_scr, *part);
    return;
  }
  if (q > 1536) {
    hipLaunchKernelGGL(k_apply_refl, dim3(ncols), dim3(256), 0, st, q, Vh, (int64_t)q, bt, Y, ldy, forward);
    HIPCK(hipGetLastError());
    return;
  }
  apply_refl_batched(st, q, ncols, 1, Vh, bt, Y, ldy, 0, forward);
}

// the register kernel over a batch of nb matrices (Vh at stride q^2, beta at
// q, Y at sY), q <= 1536
void apply_refl_batched(hipStream_t st, int q, int ncols, int nb, const z64* Vh, const double* bt, z64* Y,
                        int64_t ldy, int64_t sY, int forward) {
  if (q < 2 || ncols <= 0 || nb <= 0) return;
  if (q > 1536) fail(EAHP_EINVAL, "register reflector products: q > 1536");
  const dim3 g((ncols + 3) / 4, nb), b(256);
  const int64_t lv = q, sV = (int64_t)q * q;
  if (q <= 128) hipLaunchKernelGGL(k_apply_refl_reg<2>, g, b, 0, st, q, Vh, lv, bt, Y, ldy, ncols, forward, sV, sY);
  else if (q <= 256)
    hipLaunchKernelGGL(k_apply_refl_reg<4>, g, b, 0, st, q, Vh, lv, bt, Y, ldy, ncols, forward, sV, sY);
  else if (q <= 512)
    hipLaunchKernelGGL(k_apply_refl_reg<8>, g, b, 0, st, q, Vh, lv, bt, Y, ldy, ncols, forward, sV, sY);
  else if (q <= 1024)
    hipLaunchKernelGGL(k_apply_refl_reg<16>, g, b, 0, st, q, Vh, lv, bt, Y, ldy, ncols, forward, sV, sY);
  else hipLaunchKernelGGL(k_apply_refl_reg<24>, g, b, 0, st, q, Vh, lv, bt, Y, ldy, ncols, forward, sV, sY);
  HIPCK(hipGetLastError());
}

// Y~ (q x p, ld q) := solution of (A - s_l) y~_l = C~[:, l]; A (q x q, ld lda)
// may be destroyed.  ws grows to what the chosen kernels need.
void sylvester_tridiag(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws,
                       DevMem& part, bool store32, const BandAux* aux) {
  if (q <= 0 || p <= 0) return;
  if (q > 512) {
    sylvester_band(st, q, p, A, lda, s, Yt, ws, part, aux);
    return;
  }
  // Vh (q x q), W (3 q p), e (q), then d, beta (q each), then the scratch of
  // the reduction, then that of the blocked reflector products, then (FP32
  // storage) the single-precision copy of A
  const size_t base = sizeof(z64) * ((size_t)q * q + (size_t)3 * q * p + (size_t)q) + sizeof(double) * 2 * q + 64;
  const size_t tb = (tridiag_scratch(q) + 255) / 256 * 256;
  const bool wy = q > 512;
  const bool a32 = store32 && q > 512;
  const size_t wb = wy ? (refl_blocked_scratch(q - 1, p) + 255) / 256 * 256 : 0;
  ws.ensure(base + 256 + tb + wb + (a32 ? sizeof(c32) * (size_t)q * q : 0));
  z64* Vh = ws.as<z64>();
  z64* W = Vh + (size_t)q * q;
  z64* e = W + (size_t)3 * q * p;
  double* dd = reinterpret_cast<double*>(e + q);
  double* bt = dd + q;
  char* scr = reinterpret_cast<char*>(ws.p) + (base + 255) / 256 * 256;
  void* wscr = wy ? scr + tb : nullptr;
  if (a32) {
    c32* A32 = reinterpret_cast<c32*>(scr + tb + wb);
    convert2d(st, q, q, A, lda, A32, q);
    tridiag_reduce(st, q, A32, q, dd, e, Vh, bt, scr);
  } else {
    tridiag_reduce(st, q, A, lda, dd, e, Vh, bt, scr);
  }
  apply_refl(st, q, p, Vh, bt, Yt, q, 1, wscr, &part);
  hipLaunchKernelGGL(k_trisolve_reg, dim3((p + 63) / 64), dim3(64), 0, st, q, p, dd, e, s, Yt, (int64_t)q, W,
                     (int64_t)0);
  apply_refl(st, q, p, Vh, bt, Yt, q, 0, wscr, &part);
  HIPCK(hipGetLastError());
}

namespace {
// resident work-groups of k_tridiag_reg<NS> on the device, in matrices of
// order q: the batch of one cooperative launch
template <int NS>
int tridiag_reg_cap(int q) {
  int dev = 0, ncu = 0, per_cu = 0;
  HIPCK(hipGetDevice(&dev));
  HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_tridiag_reg<NS>, 64 * kTrWaves, 0));
  const int G = (q + kTrWaves * kTrCols - 1) / (kTrWaves * kTrCols);
  const int cap = per_cu * ncu / G;
  if (cap < 1) fail(EAHP_EDEVICE, "the tridiagonal reduction cannot be made resident");
  return cap;
}

int tridiag_batch_cap(int q) {
  if (q <= 128) return tridiag_reg_cap<2>(q);
  if (q <= 256) return tridiag_reg_cap<4>(q);
  return tridiag_reg_cap<8>(q);
}

// nb reductions in launches of up to cap matrices each (the work-groups of
// a launch are all resident); X: 2 q^2 exchange slots per matrix of a launch
template <int NS>
void tridiag_reg_batched(hipStream_t st, int q, const z64* A, int64_t lda, int64_t sA, int nb, int cap, double* dd,
                         z64* e, z64* Vh, double* bt, z64* X, int* herr) {
  const int G = (q + kTrWaves * kTrCols - 1) / (kTrWaves * kTrCols);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned long long*>(herr), (int64_t)1,
                     0ull);
  for (int k0 = 0; k0 < nb; k0 += cap) {
    const int m = std::min(cap, nb - k0);
    const int64_t nw = (int64_t)4 * q * q * m;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>(2048, (nw + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<unsigned long long*>(X), nw, kEmpty);
    int qq = q;
    int64_t la = lda, sa = sA, lv = q, sv = (int64_t)q * q, sx = 2 * (int64_t)q * q;
    const z64* Ak = A + k0 * sA;
    double* dk = dd + (int64_t)k0 * q;
    z64* ek = e + (int64_t)k0 * q;
    z64* Vk = Vh + k0 * sv;
    double* bk = bt + (int64_t)k0 * q;
    z64* Pb = X;
    z64* Cb = X + (int64_t)q * q;
    void* args[] = {&qq, &Ak, &la, &sa, &dk, &ek, &Vk, &lv, &sv, &bk, &Pb, &Cb, &sx, &herr};
    HIPCK(hipLaunchCooperativeKernel((const void*)k_tridiag_reg<NS>, dim3(G, m), dim3(64 * kTrWaves), args, 0, st));
  }
}
}  // namespace

// d_b = Re A_b[0, 0] (order 1: the matrix is its own tridiagonal form)
__global__ void k_set_d0_b(int nb, const z64* A, int64_t sA, double* d) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) d[b] = A[b * sA].x;
}

size_t sylvester_tridiag_batched_scratch(int q, int p, int nb) {
  if (q < 1 || p <= 0 || nb <= 0) return 0;
  if (q == 1) return sizeof(z64) * ((size_t)3 * p + 1) * nb + sizeof(double) * 2 * nb + 256;
  const int m = std::min(nb, tridiag_batch_cap(q));
  const size_t per = sizeof(z64) * ((size_t)q * q + (size_t)3 * q * p + q) + sizeof(double) * 2 * q;
  return per * nb + sizeof(z64) * 2 * (size_t)q * q * m + 256;
}

void sylvester_tridiag_batched(hipStream_t st, int q, int p, int nb, const z64* A, int64_t lda, int64_t sA,
                               const double* s, z64* Y, DevMem& ws) {
  if (q <= 0 || p <= 0 || nb <= 0) return;
  if (q > 512) fail(EAHP_EINVAL, "batched tridiagonal Sylvester solve: q > 512");
  ws.ensure(sylvester_tridiag_batched_scratch(q, p, nb));
  if (q == 1) {
    z64* W = ws.as<z64>() + nb;
    z64* e = W + (size_t)3 * p * nb;
    double* dd = reinterpret_cast<double*>(e + nb);
    hipLaunchKernelGGL(k_set_d0_b, dim3((nb + 63) / 64), dim3(64), 0, st, nb, A, sA, dd);
    hipLaunchKernelGGL(k_trisolve_reg, dim3((p + 63) / 64, nb), dim3(64), 0, st, 1, p, dd, e, s, Y, (int64_t)1, W,
                       (int64_t)p);
    HIPCK(hipGetLastError());
    return;
  }
  const int cap = tridiag_batch_cap(q);
  // per matrix: Vh (q^2), W (3 q p), e (q); then d and beta (q each); then the
  // exchange slots of one launch and the error flag
  z64* Vh = ws.as<z64>();
  z64* W = Vh + (size_t)q * q * nb;
  z64* e = W + (size_t)3 * q * p * nb;
  double* dd = reinterpret_cast<double*>(e + (size_t)q * nb);
  double* bt = dd + (size_t)q * nb;
  z64* X = reinterpret_cast<z64*>(bt + (size_t)q * nb);
  int* herr = reinterpret_cast<int*>(X + 2 * (size_t)q * q * std::min(nb, cap));
  {
    std::lock_guard<std::mutex> lk(coop_mutex());
    if (q <= 128) tridiag_reg_batched<2>(st, q, A, lda, sA, nb, cap, dd, e, Vh, bt, X, herr);
    else if (q <= 256) tridiag_reg_batched<4>(st, q, A, lda, sA, nb, cap, dd, e, Vh, bt, X, herr);
    else tridiag_reg_batched<8>(st, q, A, lda, sA, nb, cap, dd, e, Vh, bt, X, herr);
    int bad = 0;
    HIPCK(hipMemcpyAsync(&bad, herr, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (bad != 0) fail(EAHP_EDEVICE, "exchange wait of the tridiagonal reduction timed out");
  }
  const int64_t sY = (int64_t)q * p;
  apply_refl_batched(st, q, p, nb, Vh, bt, Y, q, sY, 1);
  hipLaunchKernelGGL(k_trisolve_reg, dim3((p + 63) / 64, nb), dim3(64), 0, st, q, p, dd, e, s, Y, (int64_t)q, W, sY);
  HIPCK(hipGetLastError());
  apply_refl_batched(st, q, p, nb, Vh, bt, Y, q, sY, 0);
}

}  // namespace eahp
