// Projected Sylvester solve of the block FOM (Algorithm 4): A Y - Y Sigma = C
// with A (q x q) and Sigma (p x p) Hermitian.  In the eigenbasis of
// Sigma = U diag(s) U^H the columns decouple into (A - s_l I) y~_l = c~_l.
// A is reduced once to Hermitian tridiagonal form A = Q T Q^H with Householder
// reflectors (a cooperative kernel over many work-groups, one grid barrier
// pair per column), after which every shifted system is a tridiagonal solve:
//
//   y~_l = Q (T - s_l I)^-1 Q^H c~_l.
//
// The result is the same Galerkin solution as with a full eigendecomposition
// of A (it is unique), at the cost of one reduction of A per FOM iteration.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>

#include "devcommon.h"
#include "kernels.h"

namespace cg = cooperative_groups;

namespace eahp {

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
__device__ void tri_reflector(int m, const z64* x_in, z64* v, double* red, double* sc, z64& alpha, double& b) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double s2 = 0;
  for (int i = tid; i < m; i += nt) {
    const z64 t = x_in ? x_in[i] : v[i];
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

// p entries of the owned columns c >= c_first: P[c - (k+1)] = b * conj(A[k+1:, c]) . v
// one wave per column, wave-level reduction
__device__ void tri_matvec(int q, int k, int c_first, int G, const z64* A, int64_t lda, const z64* v, double b,
                           z64* P) {
  const int m = q - k - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int g = blockIdx.x;
  const int c0 = c_first + ((g - c_first) % G + G) % G;
  for (int c = c0 + wave * G; c < q; c += nw * G) {
    const z64* col = A + (k + 1) + (int64_t)c * lda;
    double sx = 0, sy = 0;
    for (int r = lane; r < m; r += 64) {
      const z64 a = col[r], vr = v[r];
      sx += a.x * vr.x + a.y * vr.y;
      sy += a.x * vr.y - a.y * vr.x;
    }
    sx = warp_sum(sx);
    sy = warp_sum(sy);
    if (lane == 0) P[c - (k + 1)] = mk<double>(b * sx, b * sy);
  }
}

__global__ void __launch_bounds__(1024) k_tridiag(int q, z64* A, int64_t lda, double* d, z64* e, z64* Vh,
                                                  int64_t ldv, double* beta, z64* Pbuf) {
  extern __shared__ unsigned char smem_raw[];
  z64* v = reinterpret_cast<z64*>(smem_raw);  // q
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
    if (tid == 0) {
      d[0] = A[0].x;
      e[0] = alpha;
      beta[0] = b;
    }
  }
  tri_matvec(q, 0, 1, G, A, lda, v, b, Pbuf);
  grid.sync();
  for (int k = 0; k + 1 < q; ++k) {
    const int m = q - k - 1;
    const z64* P = Pbuf + (int64_t)(k & 1) * q;
    z64* Pn = Pbuf + (int64_t)((k + 1) & 1) * q;
    // w = p - (beta/2)(v^H p) v
    double kx = 0;
    for (int i = tid; i < m; i += nt) {
      const z64 pi = P[i];
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
        const z64 a = A[(k + 1) + (int64_t)(k + 1) * lda];
        const double u = 2.0 * (v[0].x * w[0].x + v[0].y * w[0].y);
        d[k + 1] = a.x - u;
      }
      break;
    }
    // update owned columns c >= k + 2, one wave per column
    {
      const int cf = k + 2;
      const int c0 = cf + ((g - cf) % G + G) % G;
      for (int c = c0 + wave * G; c < q; c += nw * G) {
        const int j = c - (k + 1);
        const z64 wj = w[j], vj = v[j];
        z64* col = A + (k + 1) + (int64_t)c * lda;
        for (int r = lane; r < m; r += 64) {
          const z64 vr = v[r], wr = w[r];
          const double ux = vr.x * wj.x + vr.y * wj.y + wr.x * vj.x + wr.y * vj.y;
          const double uy = vr.y * wj.x - vr.x * wj.y + wr.y * vj.x - wr.x * vj.y;
          const z64 a = col[r];
          col[r] = mk<double>(a.x - ux, a.y - uy);
        }
      }
    }
    // updated column k+1 (rows k+2..), recomputed redundantly: x = A[k+2:, k+1] - v w_0^* - w v_0^*
    const int m2 = m - 1;
    {
      const z64* colk1 = A + (k + 2) + (int64_t)(k + 1) * lda;
      const z64 w0 = w[0], v0 = v[0];
      for (int r = tid; r < m2; r += nt) {
        const z64 vr = v[r + 1], wr = w[r + 1];
        const double ux = vr.x * w0.x + vr.y * w0.y + wr.x * v0.x + wr.y * v0.y;
        const double uy = vr.y * w0.x - vr.x * w0.y + wr.y * v0.x - wr.x * v0.y;
        const z64 a = colk1[r];
        vn[r] = mk<double>(a.x - ux, a.y - uy);
      }
    }
    double dk1 = 0;
    if (tid == 0) {
      const z64 a = A[(k + 1) + (int64_t)(k + 1) * lda];
      dk1 = a.x - 2.0 * (v[0].x * w[0].x + v[0].y * w[0].y);
    }
    __syncthreads();
    // next reflector from vn (in place), then it becomes v
    tri_reflector(m2, nullptr, vn, red, sc, alpha, b);
    for (int i = tid; i < m2; i += nt) v[i] = vn[i];
    __syncthreads();
    if (g == 0) {
      for (int i = tid; i < m2; i += nt) Vh[(k + 2 + i) + (int64_t)(k + 1) * ldv] = v[i];
      if (tid == 0) {
        d[k + 1] = dk1;
        e[k + 1] = alpha;
        beta[k + 1] = b;
      }
    }
    // p of step k+1 on owned columns c >= k + 2 (already updated by this work-group)
    tri_matvec(q, k + 1, k + 2, G, A, lda, v, b, Pn);
    grid.sync();
  }
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

// (T - s_l I) z = b for every column l (in place in B), Gaussian elimination
// with partial pivoting between adjacent rows (one fill-in super-diagonal).
// T[k][k] = d_k, T[k+1][k] = e_k, T[k][k+1] = conj(e_k).  W: 3 q scratch per column.
__global__ void k_trisolve(int q, int ncols, const double* d, const z64* e, const double* s, z64* B, int64_t ldb,
                           z64* W) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= ncols) return;
  z64* b = B + (int64_t)l * ldb;
  z64* D = W + (int64_t)l * 3 * q;
  z64* U = D + q;
  z64* L = U + q;  // sub-diagonal, later the fill-in second super-diagonal
  const double sl = s[l];
  for (int i = 0; i < q; ++i) {
    D[i] = mk<double>(d[i] - sl, 0.0);
    if (i + 1 < q) {
      L[i] = e[i];
      U[i] = mk<double>(e[i].x, -e[i].y);
    }
  }
  for (int i = 0; i + 1 < q; ++i) {
    if (cabs_(D[i]) >= cabs_(L[i])) {
      const z64 f = cdiv_(L[i], D[i]);
      D[i + 1] = csub<double>(D[i + 1], cmul<double>(f, U[i]));
      b[i + 1] = csub<double>(b[i + 1], cmul<double>(f, b[i]));
      L[i] = mk<double>(0, 0);
    } else {
      const z64 f = cdiv_(D[i], L[i]);
      D[i] = L[i];
      const z64 t = D[i + 1];
      D[i + 1] = csub<double>(U[i], cmul<double>(f, t));
      if (i + 2 < q) {
        L[i] = U[i + 1];
        U[i + 1] = mk<double>(-(f.x * L[i].x - f.y * L[i].y), -(f.x * L[i].y + f.y * L[i].x));
      } else {
        L[i] = mk<double>(0, 0);
      }
      U[i] = t;
      const z64 bi = b[i];
      b[i] = b[i + 1];
      b[i + 1] = csub<double>(bi, cmul<double>(f, b[i]));
    }
  }
  b[q - 1] = cdiv_(b[q - 1], D[q - 1]);
  if (q >= 2) b[q - 2] = cdiv_(csub<double>(b[q - 2], cmul<double>(U[q - 2], b[q - 1])), D[q - 2]);
  for (int i = q - 3; i >= 0; --i) {
    z64 r = csub<double>(b[i], cmul<double>(U[i], b[i + 1]));
    r = csub<double>(r, cmul<double>(L[i], b[i + 2]));
    b[i] = cdiv_(r, D[i]);
  }
}

__global__ void k_set_d0(const z64* A, double* d) { d[0] = A[0].x; }

// Y~ (q x p, ld q) := solution of (A - s_l) y~_l = C~[:, l]; A (q x q, ld lda) is
// destroyed.  ws must hold q*q + q*3*p + 4*q complex values.
void sylvester_tridiag(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws) {
  if (q <= 0 || p <= 0) return;
  if (q > 3200) fail(EAHP_EINVAL, "projected FOM system larger than 3200");
  const size_t need = sizeof(z64) * ((size_t)q * q + (size_t)3 * q * p + 4 * (size_t)q) + sizeof(double) * 2 * q + 256;
  // P is double-buffered: 2 q entries after e (q) fit in the 4 q tail
  ws.ensure(need);
  z64* Vh = ws.as<z64>();
  z64* W = Vh + (size_t)q * q;
  z64* e = W + (size_t)3 * q * p;
  z64* P = e + q;
  double* dd = reinterpret_cast<double*>(P + 2 * q);
  double* bt = dd + q;
  if (q >= 2) {
    const size_t lds = sizeof(z64) * 3 * (size_t)q;
    HIPCK(hipFuncSetAttribute((const void*)k_tridiag, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_tridiag, 1024, lds));
    int dev = 0, ncu = 0;
    HIPCK(hipGetDevice(&dev));
    HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // one work-group per 16 columns: enough waves for the column loops, few work-groups per barrier
    const int G = std::min({std::max(1, per_cu) * ncu, ncu, std::max(1, (q + 15) / 16)});
    int qq = q;
    int64_t la = lda, lv = q;
    void* args[] = {&qq, &A, &la, &dd, &e, &Vh, &lv, &bt, &P};
    {
      // grid-synchronising kernels of concurrent streams (the serving loop)
      // could each hold part of the CUs while waiting for the rest of their
      // grid: one at a time per process, waited for before the next
      static std::mutex coop;
      std::lock_guard<std::mutex> lk(coop);
      HIPCK(hipLaunchCooperativeKernel((const void*)k_tridiag, dim3(G), dim3(1024), args, lds, st));
      HIPCK(hipStreamSynchronize(st));
    }
    hipLaunchKernelGGL(k_apply_refl, dim3(p), dim3(256), 0, st, q, Vh, (int64_t)q, bt, Yt, (int64_t)q, 1);
  } else {
    hipLaunchKernelGGL(k_set_d0, dim3(1), dim3(1), 0, st, A, dd);
  }
  hipLaunchKernelGGL(k_trisolve, dim3((p + 63) / 64), dim3(64), 0, st, q, p, dd, e, s, Yt, (int64_t)q, W);
  if (q >= 2) hipLaunchKernelGGL(k_apply_refl, dim3(p), dim3(256), 0, st, q, Vh, (int64_t)q, bt, Yt, (int64_t)q, 0);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
