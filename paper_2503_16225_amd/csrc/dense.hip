// Small dense linear algebra on the device (p x p and q x q matrices).
//
// heev      : Hermitian eigendecomposition by the cyclic Jacobi method with the
//             round-robin (circle) ordering, so that n/2 disjoint rotations are
//             applied per step; one work-group per matrix.  Used for the polar
//             factor (eq. (3.1)), the Lyapunov equation of the transport
//             (eq. (3.4)) and the projected Sylvester equations of the FOM.
// inverse   : Gauss-Jordan with partial pivoting (the p x p solve of the
//             energy-adaptive gradient, Sec. 5.2).
// pchol_inv : diagonally pivoted Cholesky of a Gram matrix with rank cut-off,
//             returning the inverse factor with the pivot permutation folded in
//             (the rank-revealing orthonormalisation of Algorithm 4).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "devcommon.h"
#include "kernels.h"

namespace cg = cooperative_groups;

namespace eahp {

// ------------------------------------------------------------------ Jacobi
__device__ __forceinline__ int rr_member(int m, int r, int np) {
  // circle method: position m of round r, players 1..np-1 rotate, 0 fixed
  return m == 0 ? 0 : ((m - 1 + r) % (np - 1)) + 1;
}

__global__ void __launch_bounds__(1024) k_heev(int n, z64* Ab, int64_t lda, int64_t sA, double* wb, int64_t sw,
                                               z64* Vb, int64_t ldv, int64_t sV, int* info) {
  extern __shared__ unsigned char smem_raw[];
  const int np = n + (n & 1);   // even number of players; index n is a dummy for odd n
  const int half = np / 2;
  z64* ph = reinterpret_cast<z64*>(smem_raw);            // half: e^{-i phi}
  double* cs = reinterpret_cast<double*>(ph + half);     // half: c
  double* sn = cs + half;                                // half: s
  double* red = sn + half;                               // 32
  int* pi = reinterpret_cast<int*>(red + 32);            // half: first of pair
  int* qi = pi + half;                                   // half: second of pair
  __shared__ int done;
  z64* A = Ab + blockIdx.x * sA;
  z64* V = Vb + blockIdx.x * sV;
  double* w = wb + blockIdx.x * sw;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    V[i + (int64_t)j * ldv] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
  }
  // Hermitise the input
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    if (i < j) {
      const z64 a = A[i + (int64_t)j * lda], b = A[j + (int64_t)i * lda];
      const z64 h = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      A[i + (int64_t)j * lda] = h;
      A[j + (int64_t)i * lda] = mk<double>(h.x, -h.y);
    } else if (i == j) {
      A[i + (int64_t)i * lda].y = 0.0;
    }
  }
  __syncthreads();
  int sweeps = 0;
  const double tol2 = (4.0 * n * 2.220446049250313e-16) * (4.0 * n * 2.220446049250313e-16);
  double prev_off = -1.0;
  for (; sweeps < 40; ++sweeps) {
    // convergence test: off-diagonal mass against the whole matrix
    double off = 0, tot = 0;
    for (int e = tid; e < n * n; e += nt) {
      const int i = e % n, j = e / n;
      const z64 a = A[i + (int64_t)j * lda];
      const double m2 = a.x * a.x + a.y * a.y;
      tot += m2;
      if (i != j) off += m2;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red + 16);
    if (tid == 0)
      done = (off <= tol2 * tot) || (tot == 0.0) || (prev_off >= 0.0 && off < 1e-20 * tot && off > 0.25 * prev_off);
    prev_off = off;
    __syncthreads();
    if (done) break;
    for (int r = 0; r < np - 1; ++r) {
      // pairs of this round and their rotations
      for (int k = tid; k < half; k += nt) {
        int a = rr_member(k, r, np), b = rr_member(np - 1 - k, r, np);
        if (a > b) { const int t = a; a = b; b = t; }
        pi[k] = a;
        qi[k] = b;
        double c = 1.0, s = 0.0;
        z64 e = mk<double>(1.0, 0.0);
        if (b < n) {
          const z64 apq = A[a + (int64_t)b * lda];
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          if (mag > 0.0) {
            const double app = A[a + (int64_t)a * lda].x, aqq = A[b + (int64_t)b * lda].x;
            const double tau = (aqq - app) / (2.0 * mag);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            e = mk<double>(apq.x / mag, -apq.y / mag);  // e^{-i phi}
          }
        }
        cs[k] = c;
        sn[k] = s;
        ph[k] = e;
      }
      __syncthreads();
      // U_k = [[c, s], [-s e, c e]] acting on columns (p, q); A <- U^H A U on 2x2 blocks
      for (int e2 = tid; e2 < half * half; e2 += nt) {
        const int P = e2 % half, Q = e2 / half;
        const int p0 = pi[P], p1 = qi[P], q0 = pi[Q], q1 = qi[Q];
        const bool vp1 = p1 < n, vq1 = q1 < n;
        z64 a00 = A[p0 + (int64_t)q0 * lda];
        z64 a01 = vq1 ? A[p0 + (int64_t)q1 * lda] : mk<double>(0, 0);
        z64 a10 = vp1 ? A[p1 + (int64_t)q0 * lda] : mk<double>(0, 0);
        z64 a11 = (vp1 && vq1) ? A[p1 + (int64_t)q1 * lda] : mk<double>(0, 0);
        // right multiply by U_Q: columns q0, q1
        const double cq = cs[Q], sq = sn[Q];
        const z64 eq = ph[Q];
        z64 b00 = cadd<double>(cscale<double>(a00, cq), cscale<double>(cmul<double>(a01, eq), -sq));
        z64 b01 = cadd<double>(cscale<double>(a00, sq), cscale<double>(cmul<double>(a01, eq), cq));
        z64 b10 = cadd<double>(cscale<double>(a10, cq), cscale<double>(cmul<double>(a11, eq), -sq));
        z64 b11 = cadd<double>(cscale<double>(a10, sq), cscale<double>(cmul<double>(a11, eq), cq));
        // left multiply by U_P^H: rows p0, p1 ; U^H = [[c, -s conj(e)], [s, c conj(e)]]
        const double cp = cs[P], sp = sn[P];
        const z64 epc = mk<double>(ph[P].x, -ph[P].y);
        z64 c00 = cadd<double>(cscale<double>(b00, cp), cscale<double>(cmul<double>(b10, epc), -sp));
        z64 c01 = cadd<double>(cscale<double>(b01, cp), cscale<double>(cmul<double>(b11, epc), -sp));
        z64 c10 = cadd<double>(cscale<double>(b00, sp), cscale<double>(cmul<double>(b10, epc), cp));
        z64 c11 = cadd<double>(cscale<double>(b01, sp), cscale<double>(cmul<double>(b11, epc), cp));
        if (P == Q && vp1) {
          c01 = mk<double>(0.0, 0.0);  // annihilated by construction
          c10 = mk<double>(0.0, 0.0);
          c00.y = 0.0;
          c11.y = 0.0;
        }
        A[p0 + (int64_t)q0 * lda] = c00;
        if (vq1) A[p0 + (int64_t)q1 * lda] = c01;
        if (vp1) A[p1 + (int64_t)q0 * lda] = c10;
        if (vp1 && vq1) A[p1 + (int64_t)q1 * lda] = c11;
      }
      // V <- V U
      for (int e2 = tid; e2 < n * half; e2 += nt) {
        const int row = e2 % n, Q = e2 / n;
        const int q0 = pi[Q], q1 = qi[Q];
        if (q1 >= n) continue;
        const double cq = cs[Q], sq = sn[Q];
        const z64 eq = ph[Q];
        const z64 v0 = V[row + (int64_t)q0 * ldv], v1 = V[row + (int64_t)q1 * ldv];
        const z64 v1e = cmul<double>(v1, eq);
        V[row + (int64_t)q0 * ldv] = cadd<double>(cscale<double>(v0, cq), cscale<double>(v1e, -sq));
        V[row + (int64_t)q1 * ldv] = cadd<double>(cscale<double>(v0, sq), cscale<double>(v1e, cq));
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += nt) w[i] = A[i + (int64_t)i * lda].x;
  if (tid == 0 && info) info[blockIdx.x] = sweeps >= 40 ? 1 : 0;
}

bool heev_dc(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V, int64_t ldv,
             int64_t sV, int batch, DevMem& scr);
bool heev_big(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V,
              int64_t ldv, int64_t sV, int batch, DevMem& scr);
bool pchol_inv_reg(hipStream_t st, int n, const z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* U,
                   int64_t ldu, DevMem& scr, bool pivot);
bool pchol_inv_big(hipStream_t st, int n, z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* U, int64_t ldu,
                   DevMem& scr, bool pivot);

void heev(hipStream_t st, int n, z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V, int64_t ldv,
          int64_t sV, int batch, int* info, DevMem& scr) {
  if (n <= 0 || batch <= 0) return;
  if (heev_dc(st, n, A, lda, sA, w, sw, V, ldv, sV, batch, scr)) return;
  if (heev_big(st, n, A, lda, sA, w, sw, V, ldv, sV, batch, scr)) return;
  // beyond the divide-and-conquer sizes: cyclic Jacobi, whose sweep limit is
  // checked here (a synchronisation on this rare path)
  const int np = n + (n & 1), half = np / 2;
  const size_t lds = (size_t)half * (2 * sizeof(int) + 2 * sizeof(double) + sizeof(z64)) + 32 * sizeof(double) + 64;
  const int nt = n <= 32 ? 256 : 1024;
  HIPCK(hipFuncSetAttribute((const void*)k_heev, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_heev, dim3(batch), dim3(nt), lds, st, n, A, lda, sA, w, sw, V, ldv, sV, info);
  HIPCK(hipGetLastError());
  std::vector<int> h(batch, 0);
  HIPCK(hipMemcpyAsync(h.data(), info, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (int b = 0; b < batch; ++b)
    if (h[b] != 0) fail(EAHP_ENOCONV, "Jacobi eigensolver did not converge in 40 sweeps");
}

// ------------------------------------------------------------------ Gauss-Jordan inverse
// work: n x 2n augmented matrix per batch entry
__global__ void __launch_bounds__(1024) k_inverse(int n, z64* Ab, int64_t lda, int64_t sA, z64* Wb, int* info) {
  __shared__ double vmax[1024];
  __shared__ int imax[1024];
  __shared__ int piv;
  __shared__ z64 pinv;
  __shared__ z64 fcol[1024];
  z64* A = Ab + blockIdx.x * sA;
  z64* W = Wb + (int64_t)blockIdx.x * n * 2 * n;  // W[i + j n], j < 2n
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = 2 * n;
  for (int e = tid; e < n * m; e += nt) {
    const int i = e % n, j = e / n;
    W[e] = j < n ? A[i + (int64_t)j * lda] : mk<double>(i == j - n ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int bad = 0;
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += nt) {
      const z64 v = W[i + (int64_t)k * n];
      const double a = v.x * v.x + v.y * v.y;
      if (a > best) { best = a; bi = i; }
    }
    vmax[tid] = best;
    imax[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double o = vmax[tid + s];
        const int oi = imax[tid + s];
        if (o > vmax[tid] || (o == vmax[tid] && oi < imax[tid])) { vmax[tid] = o; imax[tid] = oi; }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int ib = imax[0] < n ? imax[0] : k;
      piv = ib;
      const z64 d = W[ib + (int64_t)k * n];
      const double den = d.x * d.x + d.y * d.y;
      pinv = den > 0 ? mk<double>(d.x / den, -d.y / den) : mk<double>(0, 0);
    }
    __syncthreads();
    if (pinv.x == 0.0 && pinv.y == 0.0) bad = 1;
    const int pr = piv;
    // columns 0..k-1 of the A part are already unit vectors; all others take part
    const int width = m - k;
    if (pr != k)
      for (int t = tid; t < width; t += nt) {
        const int j = k + t;
        const z64 tv = W[k + (int64_t)j * n];
        W[k + (int64_t)j * n] = W[pr + (int64_t)j * n];
        W[pr + (int64_t)j * n] = tv;
      }
    __syncthreads();
    for (int t = tid; t < width; t += nt) {
      const int j = k + t;
      W[k + (int64_t)j * n] = cmul<double>(W[k + (int64_t)j * n], pinv);
    }
    for (int i = tid; i < n; i += nt) fcol[i] = W[i + (int64_t)k * n];
    __syncthreads();
    for (int e = tid; e < n * width; e += nt) {
      const int i = e % n, t = e / n;
      if (i == k) continue;
      const int j = k + t;
      const z64 f = fcol[i];
      W[i + (int64_t)j * n] = csub<double>(W[i + (int64_t)j * n], cmul<double>(f, W[k + (int64_t)j * n]));
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    A[i + (int64_t)j * lda] = W[i + (int64_t)(j + n) * n];
  }
  if (tid == 0 && info) info[blockIdx.x] = bad;
}

// In-place Gauss-Jordan (the sweep at each pivot) for n <= 128 with the matrix
// in registers: thread t owns row t/8 and the 16 columns congruent to t mod 8.
// Column k is eliminated at step k with the unused row of largest modulus in
// it (ties: the smaller row index); rows are exchanged only logically, so the
// swept matrix B holds the inverse as inv(A)[pos(r)][piv(j)] = B[r][j], with
// piv(k) the pivot row of step k and pos its inverse.  Per step: the pivot
// candidates of each wave (a shuffle reduction over its 8 rows) meet in LDS,
// every thread picks the winner itself, the pivot row is scaled into LDS and
// every other row takes its rank-1 update.
__global__ void __launch_bounds__(1024) k_inverse_reg(int n, z64* Ab, int64_t lda, int64_t sA, int* info) {
  __shared__ double cv[16];
  __shared__ int ci[16];
  __shared__ z64 cz[16];
  __shared__ z64 prow[128];
  __shared__ int prk[128], pos[128];
  z64* A = Ab + blockIdx.x * sA;
  const int t = threadIdx.x, rr = t >> 3, cg = t & 7, lane = t & 63, wv = t >> 6;
  const int ncg = n - cg;  // column cg + 8 m exists while 8 m < ncg
  d16 ar, ai;              // row rr, columns cg + 8 m (real and imaginary parts)
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const z64 v = (rr < n && 8 * m < ncg) ? A[rr + (int64_t)(cg + 8 * m) * lda] : mk<double>(0.0, 0.0);
    ar[m] = v.x;
    ai[m] = v.y;
  }
  bool used = rr >= n;
  int bad = 0;
  for (int k = 0; k < n; ++k) {
    const int km = __builtin_amdgcn_readfirstlane(k >> 3);
    const bool mine = cg == (k & 7);  // this lane holds column k (in slot km)
    const z64 ak = mk<double>(ar[km], ai[km]);
    // candidate of this wave: the largest |a_rk| over its unused rows
    double val = (mine && !used) ? ak.x * ak.x + ak.y * ak.y : -1.0;
    int row = (mine && !used) ? rr : 1 << 20;
    wave_argmax(val, row);
    if (lane == 0) {
      cv[wv] = val;
      ci[wv] = row;
    }
    if (mine && rr == row) cz[wv] = ak;
    // entry of column k in this thread's row, from the lane of the row that holds it
    const int src = (lane & ~7) | (k & 7);
    const z64 f = mk<double>(__shfl(ak.x, src, 64), __shfl(ak.y, src, 64));
    __syncthreads();
    double best = lane < 16 ? cv[lane] : -2.0;
    int pr = lane < 16 ? ci[lane] : 1 << 20;
    row16_argmax(best, pr);
    pr = __builtin_amdgcn_readlane(pr, 0);
    const z64 pz = cz[pr >> 3];
    const double den = pz.x * pz.x + pz.y * pz.y;
    if (!(den > 0)) bad = 1;
    const z64 pinv = den > 0 ? mk<double>(pz.x / den, -pz.y / den) : mk<double>(0.0, 0.0);
    const bool piv = rr == pr;
    if (piv) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        prow[cg + 8 * m] = mk<double>(ar[m] * pinv.x - ai[m] * pinv.y, ar[m] * pinv.y + ai[m] * pinv.x);
        ar[m] = 0.0;
        ai[m] = 0.0;
      }
      if (mine) prow[k] = pinv;
      used = true;
      if (cg == 0) {
        prk[k] = pr;
        pos[pr] = k;
      }
    }
    __syncthreads();
    // every row: a_rj + g prow_j with g = -a_rk (1 on the pivot row, whose a is
    // zeroed above); then column k of the other rows becomes -a_rk pinv
    const z64 g = piv ? mk<double>(1.0, 0.0) : mk<double>(-f.x, -f.y);
#pragma unroll
    for (int mb = 0; mb < 16; mb += 4) {
      z64 pw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pw[u] = prow[cg + 8 * (mb + u)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int m = mb + u;
        ar[m] = fma(g.x, pw[u].x, fma(-g.y, pw[u].y, ar[m]));
        ai[m] = fma(g.x, pw[u].y, fma(g.y, pw[u].x, ai[m]));
      }
    }
    {
      const bool fix = mine && !piv;
      const double nr = fix ? -(f.x * pinv.x - f.y * pinv.y) : ar[km];
      const double ni = fix ? -(f.x * pinv.y + f.y * pinv.x) : ai[km];
      ar[km] = nr;
      ai[km] = ni;
    }
  }
  __syncthreads();
  if (rr < n) {
    const int r = pos[rr];
#pragma unroll
    for (int m = 0; m < 16; ++m)
      if (8 * m < ncg) A[r + (int64_t)prk[cg + 8 * m] * lda] = mk<double>(ar[m], ai[m]);
  }
  if (t == 0 && info) info[blockIdx.x] = bad;
}

// Gauss-Jordan on [A | I] (n x 2n, column-major in W) with partial pivoting
// for n > 128: the columns are spread over the work-groups of a cooperative
// grid (column c to group c mod G), one grid barrier per step.  In step k
// every group reads column k (nobody writes it in step k: once its pivot is
// chosen, left column k is never read again), chooses the same pivot row
// (largest modulus among the rows not yet pivots, ties to the smallest index)
// and eliminates column k from its own columns j > k.  Row p_k of the right
// half then holds row k of A^-1.
__global__ void __launch_bounds__(256) k_inverse_coop(int n, z64* A, int64_t lda, z64* W, int* info) {
  extern __shared__ unsigned char smem_raw[];
  z64* colk = reinterpret_cast<z64*>(smem_raw);  // n
  int* used = reinterpret_cast<int*>(colk + n);   // n
  int* prow = used + n;                           // n
  z64* prv = reinterpret_cast<z64*>(prow + n + (n & 1));  // own columns
  __shared__ double cv[4];
  __shared__ int ci[4];
  cg::grid_group grid = cg::this_grid();
  const int G = gridDim.x, g = blockIdx.x, t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  const int m = 2 * n;
  for (int j = g; j < m; j += G)
    for (int i = t; i < n; i += nt)
      W[i + (int64_t)j * n] = j < n ? A[i + (int64_t)j * lda] : mk<double>(i == j - n ? 1.0 : 0.0, 0.0);
  for (int i = t; i < n; i += nt) used[i] = 0;
  int bad = 0;
  grid.sync();
  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int br = 1 << 20;
    for (int i = t; i < n; i += nt) {
      const z64 v = W[i + (int64_t)k * n];
      colk[i] = v;
      const double a = v.x * v.x + v.y * v.y;
      if (!used[i] && a > best) {
        best = a;
        br = i;
      }
    }
    wave_argmax(best, br);
    if (lane == 0) {
      cv[wv] = best;
      ci[wv] = br;
    }
    __syncthreads();
    best = cv[0];
    br = ci[0];
    for (int w = 1; w < (nt >> 6); ++w) argmax_merge(best, br, cv[w], ci[w]);
    const int p = br;
    const z64 pz = colk[p];
    const double den = pz.x * pz.x + pz.y * pz.y;
    if (!(den > 0)) bad = 1;
    const z64 pinv = den > 0 ? mk<double>(pz.x / den, -pz.y / den) : mk<double>(0.0, 0.0);
    // scaled pivot-row entries of the own columns j > k
    const int j0 = k + 1 + ((g - (k + 1)) % G + G) % G;
    for (int j = j0 + t * G; j < m; j += nt * G) prv[(j - j0) / G] = cmul<double>(W[p + (int64_t)j * n], pinv);
    __syncthreads();
    const int nown = j0 < m ? (m - j0 + G - 1) / G : 0;
    for (int i = t; i < n; i += nt) {
      const z64 f = colk[i];
      for (int c = 0; c < nown; ++c) {
        z64* wc = W + (int64_t)(j0 + c * G) * n;
        const z64 pr = prv[c];
        if (i == p) wc[i] = pr;
        else wc[i] = csub<double>(wc[i], cmul<double>(f, pr));
      }
    }
    if (t == 0) {
      used[p] = 1;
      prow[k] = p;
    }
    grid.sync();
  }
  // A^-1[k][j] = W[p_k][n + j] for the own right-half columns
  for (int j = g; j < n; j += G)
    for (int k = t; k < n; k += nt) A[k + (int64_t)j * lda] = W[prow[k] + (int64_t)(n + j) * n];
  if (g == 0 && t == 0 && info) info[0] = bad;
}

void inverse(hipStream_t st, int n, z64* A, int64_t lda, int64_t sA, z64* work, int batch, int* info) {
  if (n <= 0 || batch <= 0) return;
  if (n > 1024) fail(EAHP_EINVAL, "inverse: n > 1024");
  if (n <= 128) {
    hipLaunchKernelGGL(k_inverse_reg, dim3(batch), dim3(1024), 0, st, n, A, lda, sA, info);
    HIPCK(hipGetLastError());
    return;
  }
  int dev = 0, ncu = 0;
  HIPCK(hipGetDevice(&dev));
  HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // about 8 columns of [A | I] per work-group, at most one work-group per CU
  const int G = std::max(1, std::min(ncu, (2 * n + 7) / 8));
  const int own = (2 * n + G - 1) / G + 1;
  const size_t lds = sizeof(z64) * n + sizeof(int) * (2 * n + 2) + sizeof(z64) * own + 64;
  HIPCK(hipFuncSetAttribute((const void*)k_inverse_coop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_inverse_coop, 256, lds));
  if (per_cu < 1) fail(EAHP_EDEVICE, "the inverse cannot be made resident");
  std::lock_guard<std::mutex> lk(coop_mutex());
  for (int b = 0; b < batch; ++b) {
    int nn = n;
    z64* Ab = A + b * sA;
    int64_t la = lda;
    z64* Wb = work + (int64_t)b * 2 * n * n;
    int* ib = info ? info + b : nullptr;
    void* args[] = {&nn, &Ab, &la, &Wb, &ib};
    HIPCK(hipLaunchCooperativeKernel((const void*)k_inverse_coop, dim3(G), dim3(256), args, lds, st));
  }
  HIPCK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ pivoted Cholesky
// G (n x n Hermitian PSD) is overwritten by the pivoted factor.  Outputs
// Uinv (n x r, ld ldu): row piv[k] holds row k of L^-H, other rows zero.
__global__ void __launch_bounds__(1024) k_pchol(int n, z64* G, int64_t ldg, double tol, int* pivout, int* rank,
                                                z64* Uinv, int64_t ldu, int* info, int pivot) {
  extern __shared__ unsigned char smem_raw[];
  int* perm = reinterpret_cast<int*>(smem_raw);  // n
  __shared__ int rk, pk;
  __shared__ double d0;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) perm[i] = i;
  // Hermitise
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    if (i < j) {
      const z64 a = G[i + (int64_t)j * ldg], b = G[j + (int64_t)i * ldg];
      const z64 h = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      G[i + (int64_t)j * ldg] = h;
      G[j + (int64_t)i * ldg] = mk<double>(h.x, -h.y);
    }
  }
  if (tid == 0) { rk = n; d0 = -1.0; }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      double best = -1.0;
      int b = k;
      if (pivot) {
        for (int i = k; i < n; ++i) {
          const double v = G[i + (int64_t)i * ldg].x;
          if (v > best) { best = v; b = i; }
        }
      } else {
        best = G[k + (int64_t)k * ldg].x;
      }
      if (k == 0) d0 = best;
      pk = b;
      if (!(best > tol * d0) || !(best > 0.0)) { rk = k; }
    }
    __syncthreads();
    if (rk == k) break;
    const int b = pk;
    if (b != k) {
      // symmetric swap of rows/cols k and b
      for (int j = tid; j < n; j += nt) {
        const z64 t = G[k + (int64_t)j * ldg];
        G[k + (int64_t)j * ldg] = G[b + (int64_t)j * ldg];
        G[b + (int64_t)j * ldg] = t;
      }
      __syncthreads();
      for (int i = tid; i < n; i += nt) {
        const z64 t = G[i + (int64_t)k * ldg];
        G[i + (int64_t)k * ldg] = G[i + (int64_t)b * ldg];
        G[i + (int64_t)b * ldg] = t;
      }
      if (tid == 0) { const int t = perm[k]; perm[k] = perm[b]; perm[b] = t; }
      __syncthreads();
    }
    const double lkk = sqrt(G[k + (int64_t)k * ldg].x);
    __syncthreads();
    // column k of L: L_ik = G_ik / lkk for i > k
    for (int i = k + 1 + tid; i < n; i += nt) G[i + (int64_t)k * ldg] = cscale<double>(G[i + (int64_t)k * ldg], 1.0 / lkk);
    __syncthreads();
    if (tid == 0) G[k + (int64_t)k * ldg] = mk<double>(lkk, 0.0);
    // Schur complement on the trailing lower triangle (and its mirror)
    for (int e = tid; e < (n - k - 1) * (n - k - 1); e += nt) {
      const int i = k + 1 + e % (n - k - 1), j = k + 1 + e / (n - k - 1);
      if (i < j) continue;
      const z64 li = G[i + (int64_t)k * ldg], lj = G[j + (int64_t)k * ldg];
      const z64 upd = cmul<double>(li, mk<double>(lj.x, -lj.y));
      const z64 v = csub<double>(G[i + (int64_t)j * ldg], upd);
      G[i + (int64_t)j * ldg] = v;
      if (i != j) G[j + (int64_t)i * ldg] = mk<double>(v.x, -v.y);
      else G[i + (int64_t)i * ldg].y = 0.0;
    }
    __syncthreads();
  }
  const int r = rk;
  // L^-1 (r x r lower) by forward substitution, one column per thread, written
  // into the strict upper part scratch: store L^-1 column j in Uinv rows as we go
  for (int e = tid; e < n * r; e += nt) Uinv[(e % n) + (int64_t)(e / n) * ldu] = mk<double>(0, 0);
  __syncthreads();
  for (int j = tid; j < r; j += nt) {
    // solve L x = e_j, x_i = 0 for i < j; write conj(x_i) to Uinv[perm[j]... ] later
    // x stored temporarily in Uinv column j, rows 0..r-1 (unpermuted)
    z64* x = Uinv + (int64_t)j * ldu;
    for (int i = j; i < r; ++i) {
      z64 s = mk<double>(i == j ? 1.0 : 0.0, 0.0);
      for (int m = j; m < i; ++m) s = csub<double>(s, cmul<double>(G[i + (int64_t)m * ldg], x[m]));
      x[i] = cscale<double>(s, 1.0 / G[i + (int64_t)i * ldg].x);
    }
  }
  __syncthreads();
  // (L^-H)[k][j] = conj((L^-1)[j][k]);  Uinv[perm[k]][j] = (L^-H)[k][j] for k <= j
  // current Uinv column c holds (L^-1)[:, c]; build the result in place column by column
  // using a register copy per element (each (k, j) read once then written once).
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int k = e % r, j = e / r;
    // read (L^-1)[j][k] = Uinv[j + k ldu]
    const z64 v = (k <= j) ? Uinv[j + (int64_t)k * ldu] : mk<double>(0, 0);
    G[k + (int64_t)j * ldg] = mk<double>(v.x, -v.y);  // G now holds L^-H (r x r, upper)
  }
  __syncthreads();
  for (int e = tid; e < n * r; e += nt) Uinv[(e % n) + (int64_t)(e / n) * ldu] = mk<double>(0, 0);
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int k = e % r, j = e / r;
    Uinv[perm[k] + (int64_t)j * ldu] = G[k + (int64_t)j * ldg];
  }
  if (tid == 0) {
    *rank = r;
    if (info) *info = 0;
  }
  for (int i = tid; i < n; i += nt) pivout[i] = perm[i];
}

void pchol_inv(hipStream_t st, int n, z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* Uinv, int64_t ldu,
               int* info, DevMem& scr, bool pivot) {
  if (n <= 0) return;
  if (pchol_inv_reg(st, n, G, ldg, tol, piv, rank, Uinv, ldu, scr, pivot)) return;
  if (pchol_inv_big(st, n, G, ldg, tol, piv, rank, Uinv, ldu, scr, pivot)) return;
  const size_t lds = (size_t)n * sizeof(int) + 64;
  HIPCK(hipFuncSetAttribute((const void*)k_pchol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_pchol, dim3(1), dim3(n <= 64 ? 256 : 1024), lds, st, n, G, ldg, tol, piv, rank, Uinv, ldu,
                     info, pivot ? 1 : 0);
  HIPCK(hipGetLastError());
}

// ------------------------------------------------------------------ elementwise helpers
__global__ void k_sylv_divide(int q, int p, const double* w, const double* s, z64* Y, int64_t ldy) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q * p; e += gridDim.x * blockDim.x) {
    const int i = e % q, l = e / q;
    const double d = w[i] - s[l];
    Y[i + (int64_t)l * ldy] = cscale<double>(Y[i + (int64_t)l * ldy], 1.0 / d);
  }
}
void sylv_divide(hipStream_t st, int q, int p, const double* w, const double* s, z64* Y, int64_t ldy) {
  if (q * p <= 0) return;
  hipLaunchKernelGGL(k_sylv_divide, dim3(std::min(1024, (q * p + 255) / 256)), dim3(256), 0, st, q, p, w, s, Y, ldy);
  HIPCK(hipGetLastError());
}

// D = Omega(M) - M: zero below the diagonal, -conj(M_ji) - M_ij above, -Re M_jj on it
__global__ void k_qr_omega_minus(int p, const z64* Mb, int64_t ldm, int64_t sM, z64* Db, int64_t ldd, int64_t sD) {
  const z64* M = Mb + blockIdx.y * sM;
  z64* D = Db + blockIdx.y * sD;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e % p, j = e / p;
    const z64 m = M[i + (int64_t)j * ldm];
    z64 d;
    if (i > j) {
      d = mk<double>(0.0, 0.0);
    } else if (i == j) {
      d = mk<double>(-m.x, 0.0);
    } else {
      const z64 t = M[j + (int64_t)i * ldm];
      d = mk<double>(-t.x - m.x, t.y - m.y);
    }
    D[i + (int64_t)j * ldd] = d;
  }
}
void qr_omega_minus(hipStream_t st, int p, const z64* M, int64_t ldm, int64_t sM, z64* D, int64_t ldd, int64_t sD,
                    int batch) {
  hipLaunchKernelGGL(k_qr_omega_minus, dim3(std::min(1024, (p * p + 255) / 256), batch), dim3(256), 0, st, p, M, ldm,
                     sM, D, ldd, sD);
  HIPCK(hipGetLastError());
}

__global__ void k_lyap_divide(int p, const double* db, z64* Xb, int64_t ldx, int64_t sd, int64_t sX) {
  const double* d = db + blockIdx.y * sd;
  z64* X = Xb + blockIdx.y * sX;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int a = e % p, b = e / p;
    X[a + (int64_t)b * ldx] = cscale<double>(X[a + (int64_t)b * ldx], 1.0 / (sqrt(d[a]) + sqrt(d[b])));
  }
}
void lyap_divide(hipStream_t st, int p, const double* d, z64* X, int64_t ldx, int batch, int64_t sd, int64_t sX) {
  hipLaunchKernelGGL(k_lyap_divide, dim3(std::min(1024, (p * p + 255) / 256), batch), dim3(256), 0, st, p, d, X, ldx,
                     sd, sX);
  HIPCK(hipGetLastError());
}

// M = V diag(d^e) V^H
__global__ void k_spectral(int p, const z64* Vb, int64_t ldv, int64_t sV, const double* db, int64_t sd, double ex,
                           z64* Mb, int64_t ldm, int64_t sM) {
  const z64* V = Vb + blockIdx.y * sV;
  const double* d = db + blockIdx.y * sd;
  z64* M = Mb + blockIdx.y * sM;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e % p, j = e / p;
    double sx = 0, sy = 0;
    for (int k = 0; k < p; ++k) {
      const double f = (ex == 0.5) ? sqrt(d[k]) : (ex == -0.5 ? 1.0 / sqrt(d[k]) : pow(d[k], ex));
      const z64 a = V[i + (int64_t)k * ldv], b = V[j + (int64_t)k * ldv];
      // a * f * conj(b)
      sx += f * (a.x * b.x + a.y * b.y);
      sy += f * (a.y * b.x - a.x * b.y);
    }
    M[i + (int64_t)j * ldm] = mk<double>(sx, sy);
  }
}
// Inverse square root of S = V (diag(d) + Dt) V^H to first order in the
// Hermitian perturbation Dt (given in the eigenbasis V of the unperturbed
// part, d = 1 + tau^2 w): Mt = diag(d^-1/2) - Dt o K with
// K_ij = 1 / (s_i s_j (s_i + s_j)), s = d^1/2 (the divided difference of
// x^-1/2 at d_i, d_j).  Writes d and Mt; the caller forms V Mt V^H.
__global__ void k_polar_fo(int p, const double* wb, int64_t sw, double tau, const z64* Dtb, int64_t sD, double* db,
                           z64* Mtb, int64_t sM) {
  const double* w = wb + blockIdx.y * sw;
  const z64* Dt = Dtb + blockIdx.y * sD;
  double* d = db + blockIdx.y * sw;
  z64* Mt = Mtb + blockIdx.y * sM;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e % p, j = e / p;
    const double di = 1.0 + tau * tau * w[i], dj = 1.0 + tau * tau * w[j];
    const double si = sqrt(di), sj = sqrt(dj);
    const double k = 1.0 / (si * sj * (si + sj));
    z64 m = cscale<double>(Dt[i + (int64_t)j * p], -k);
    if (i == j) {
      m.x += 1.0 / si;
      m.y = 0.0;
      d[i] = di;
    }
    Mt[i + (int64_t)j * p] = m;
  }
}
void polar_first_order(hipStream_t st, int p, const double* w, double tau, const z64* Dt, double* d, z64* Mt,
                       int batch) {
  hipLaunchKernelGGL(k_polar_fo, dim3(std::min(1024, (p * p + 255) / 256), batch), dim3(256), 0, st, p, w,
                     (int64_t)p, tau, Dt, (int64_t)p * p, d, Mt, (int64_t)p * p);
  HIPCK(hipGetLastError());
}

__global__ void k_affine(int n, const double* x, double a, double b, double* y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] = a + b * x[i];
}
void affine(hipStream_t st, int n, const double* x, double a, double b, double* y) {
  hipLaunchKernelGGL(k_affine, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0, st, n, x, a, b, y);
  HIPCK(hipGetLastError());
}

void spectral_fn(hipStream_t st, int p, const z64* V, int64_t ldv, int64_t sV, const double* d, int64_t sd, double e,
                 z64* M, int64_t ldm, int64_t sM, int batch) {
  hipLaunchKernelGGL(k_spectral, dim3(std::min(1024, (p * p + 255) / 256), batch), dim3(256), 0, st, p, V, ldv, sV, d,
                     sd, e, M, ldm, sM);
  HIPCK(hipGetLastError());
}

__global__ void k_hermitize(int p, z64* Mb, int64_t ldm, int64_t sM) {
  z64* M = Mb + blockIdx.y * sM;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e % p, j = e / p;
    if (i < j) {
      const z64 a = M[i + (int64_t)j * ldm], b = M[j + (int64_t)i * ldm];
      const z64 h = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      M[i + (int64_t)j * ldm] = h;
      M[j + (int64_t)i * ldm] = mk<double>(h.x, -h.y);
    } else if (i == j) {
      M[i + (int64_t)i * ldm].y = 0.0;
    }
  }
}
void hermitize(hipStream_t st, int p, z64* M, int64_t ldm, int64_t sM, int batch) {
  hipLaunchKernelGGL(k_hermitize, dim3(std::min(1024, (p * p + 255) / 256), batch), dim3(256), 0, st, p, M, ldm, sM);
  HIPCK(hipGetLastError());
}

__global__ void k_add_diag(int p, z64* Mb, int64_t ldm, int64_t sM, double v) {
  z64* M = Mb + blockIdx.y * sM;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p; i += gridDim.x * blockDim.x) M[i + (int64_t)i * ldm].x += v;
}
void add_diag(hipStream_t st, int p, z64* M, int64_t ldm, int64_t sM, double v, int batch) {
  hipLaunchKernelGGL(k_add_diag, dim3(1, batch), dim3(256), 0, st, p, M, ldm, sM, v);
  HIPCK(hipGetLastError());
}

__global__ void k_set_identity(int p, z64* M, int64_t ldm) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p * p; e += gridDim.x * blockDim.x) {
    const int i = e % p, j = e / p;
    M[i + (int64_t)j * ldm] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
  }
}
void set_identity(hipStream_t st, int p, z64* M, int64_t ldm) {
  hipLaunchKernelGGL(k_set_identity, dim3(std::min(1024, (p * p + 255) / 256)), dim3(256), 0, st, p, M, ldm);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
