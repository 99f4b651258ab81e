// LDS-resident small dense kernels for n <= 128 (complex128):
//
// k_jacobi_lds : cyclic Jacobi on a Hermitian matrix held as a packed lower
//                triangle in LDS (n(n+1)/2 values, 132 KB at n = 128); the
//                rotations of every round are logged to global memory.
// k_rot_apply  : V = product of the logged rotations, rows of V split over
//                work-groups and kept in LDS while all rounds are replayed.
// k_pchol_lds  : diagonally pivoted Cholesky with rank cut-off and in-place
//                inversion of the factor, in the packed LDS triangle.
#include "devcommon.h"
#include "kernels.h"

namespace eahp {

// packed lower triangle: (i, j), i >= j, at i (i + 1) / 2 + j
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }
__device__ __forceinline__ z64 pget(const z64* P, int i, int j) {
  if (i >= j) return P[pk(i, j)];
  const z64 v = P[pk(j, i)];
  return mk<double>(v.x, -v.y);
}
__device__ __forceinline__ void pset(z64* P, int i, int j, z64 v) {
  if (i >= j) P[pk(i, j)] = v;
  else P[pk(j, i)] = mk<double>(v.x, -v.y);
}

__device__ __forceinline__ int rr_slot(int m, int r, int np) { return m == 0 ? 0 : ((m - 1 + r) % (np - 1)) + 1; }

struct Rot {
  double c, s;
  z64 e;  // e^{-i phi}
};

constexpr int kRing = 8;  // rounds of rotations buffered in LDS before a flush to global memory

// One matrix per work-group.  A (n x n, lda) is read (Hermitian part) and its
// eigenvalues written to w; rotations to log[batch][round][pair]; the number of
// rounds performed to nrounds[batch].
__global__ void __launch_bounds__(1024) k_jacobi_lds(int n, const z64* Ab, int64_t lda, int64_t sA, double* wb,
                                                     int64_t sw, Rot* logb, int64_t slog, int max_rounds,
                                                     int* nrounds) {
  extern __shared__ unsigned char smem_raw[];
  const int np = n + (n & 1), half = np / 2;
  const int nblk = half * (half + 1) / 2;
  z64* P = reinterpret_cast<z64*>(smem_raw);                   // n(n+1)/2
  Rot* ring = reinterpret_cast<Rot*>(P + n * (n + 1) / 2);     // kRing x half
  int* pa = reinterpret_cast<int*>(ring + kRing * half);       // half
  int* pb = pa + half;                                         // half
  unsigned short* bq = reinterpret_cast<unsigned short*>(pb + half);  // nblk: (Pp, Q) pairs with Pp <= Q
  __shared__ double red[32];
  __shared__ int done;
  const z64* A = Ab + blockIdx.x * sA;
  double* w = wb + blockIdx.x * sw;
  Rot* log = logb + blockIdx.x * slog;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ntri = n * (n + 1) / 2;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    if (i > j) {
      const z64 a = A[i + (int64_t)j * lda], b = A[j + (int64_t)i * lda];
      P[pk(i, j)] = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    } else if (i == j) {
      P[pk(i, i)] = mk<double>(A[i + (int64_t)i * lda].x, 0.0);
    }
  }
  // block table: entry Q (Q + 1) / 2 + Pp holds (Pp, Q)
  for (int Q = tid; Q < half; Q += nt)
    for (int Pp = 0; Pp <= Q; ++Pp) {
      bq[2 * (Q * (Q + 1) / 2 + Pp)] = (unsigned short)Pp;
      bq[2 * (Q * (Q + 1) / 2 + Pp) + 1] = (unsigned short)Q;
    }
  __syncthreads();
  int rounds = 0;
  // stop at the rounding floor: off-diagonal mass below (4 n eps)^2 of the
  // total, or no longer shrinking once below 1e-20 of it
  const double tol2 = (4.0 * n * 2.220446049250313e-16) * (4.0 * n * 2.220446049250313e-16);
  double prev_off = -1.0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i) {
      // row i of the packed triangle: entries pk(i, 0..i)
      const int base = i * (i + 1) / 2;
      for (int j = tid; j <= i; j += nt) {
        const z64 a = P[base + j];
        const double m2 = a.x * a.x + a.y * a.y;
        if (i == j) tot += m2;
        else {
          off += 2.0 * m2;
          tot += 2.0 * m2;
        }
      }
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red + 16);
    if (tid == 0)
      done = (off <= tol2 * tot) || (tot == 0.0) || (rounds + np - 1 > max_rounds) ||
             (prev_off >= 0.0 && off < 1e-20 * tot && off > 0.25 * prev_off);
    prev_off = off;
    __syncthreads();
    if (done) break;
    for (int r = 0; r < np - 1; ++r) {
      Rot* rot = ring + (rounds % kRing) * half;
      for (int k = tid; k < half; k += nt) {
        int a = rr_slot(k, r, np), b = rr_slot(np - 1 - k, r, np);
        if (a > b) { const int t = a; a = b; b = t; }
        pa[k] = a;
        pb[k] = b;
        Rot R{1.0, 0.0, mk<double>(1.0, 0.0)};
        if (b < n) {
          const z64 apq = pget(P, a, b);
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          if (mag > 0.0) {
            const double app = P[pk(a, a)].x, aqq = P[pk(b, b)].x;
            const double tau = (aqq - app) / (2.0 * mag);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            R.c = 1.0 / sqrt(1.0 + t * t);
            R.s = t * R.c;
            R.e = mk<double>(apq.x / mag, -apq.y / mag);
          }
        }
        rot[k] = R;
      }
      __syncthreads();
      // A <- U^H A U on the 2x2 blocks (P <= Q), U_k = [[c, s], [-s e, c e]]
      for (int e2 = tid; e2 < nblk; e2 += nt) {
        const int Pp = bq[2 * e2], Q = bq[2 * e2 + 1];
        const int p0 = pa[Pp], p1 = pb[Pp], q0 = pa[Q], q1 = pb[Q];
        const bool vp1 = p1 < n, vq1 = q1 < n;
        const z64 a00 = pget(P, p0, q0);
        const z64 a01 = vq1 ? pget(P, p0, q1) : mk<double>(0, 0);
        const z64 a10 = vp1 ? pget(P, p1, q0) : mk<double>(0, 0);
        const z64 a11 = (vp1 && vq1) ? pget(P, p1, q1) : mk<double>(0, 0);
        const Rot RQ = rot[Q], RP = rot[Pp];
        const z64 b00 = cadd<double>(cscale<double>(a00, RQ.c), cscale<double>(cmul<double>(a01, RQ.e), -RQ.s));
        const z64 b01 = cadd<double>(cscale<double>(a00, RQ.s), cscale<double>(cmul<double>(a01, RQ.e), RQ.c));
        const z64 b10 = cadd<double>(cscale<double>(a10, RQ.c), cscale<double>(cmul<double>(a11, RQ.e), -RQ.s));
        const z64 b11 = cadd<double>(cscale<double>(a10, RQ.s), cscale<double>(cmul<double>(a11, RQ.e), RQ.c));
        const z64 epc = mk<double>(RP.e.x, -RP.e.y);
        z64 c00 = cadd<double>(cscale<double>(b00, RP.c), cscale<double>(cmul<double>(b10, epc), -RP.s));
        z64 c01 = cadd<double>(cscale<double>(b01, RP.c), cscale<double>(cmul<double>(b11, epc), -RP.s));
        z64 c10 = cadd<double>(cscale<double>(b00, RP.s), cscale<double>(cmul<double>(b10, epc), RP.c));
        z64 c11 = cadd<double>(cscale<double>(b01, RP.s), cscale<double>(cmul<double>(b11, epc), RP.c));
        if (Pp == Q) {
          // diagonal block: (p0,p0), (p1,p1) real; (p1,p0) annihilated by the rotation
          c00.y = 0.0;
          P[pk(p0, p0)] = c00;
          if (vp1) {
            c11.y = 0.0;
            P[pk(p1, p1)] = c11;
            P[pk(p1, p0)] = mk<double>(0.0, 0.0);
          }
        } else {
          pset(P, p0, q0, c00);
          if (vq1) pset(P, p0, q1, c01);
          if (vp1) pset(P, p1, q0, c10);
          if (vp1 && vq1) pset(P, p1, q1, c11);
        }
      }
      ++rounds;
      if (rounds % kRing == 0) {
        // flush the ring (its stores are waited on only at the next barrier)
        Rot* dst = log + (int64_t)(rounds - kRing) * half;
        for (int e = tid; e < kRing * half; e += nt) dst[e] = ring[e];
      }
      __syncthreads();
    }
  }
  if (rounds % kRing) {
    const int first = rounds - rounds % kRing;
    Rot* dst = log + (int64_t)first * half;
    for (int e = tid; e < (rounds % kRing) * half; e += nt) dst[e] = ring[e];
  }
  for (int i = tid; i < n; i += nt) w[i] = P[pk(i, i)].x;
  if (tid == 0) nrounds[blockIdx.x] = rounds;
}

// V (n x n, ldv) = I * U_round0 * U_round1 * ...; grid (row blocks, batch).
// Rotations are staged kRing rounds at a time in LDS.
__global__ void __launch_bounds__(256) k_rot_apply(int n, int rows_per_wg, const Rot* logb, int64_t slog,
                                                   const int* nrounds, z64* Vb, int64_t ldv, int64_t sV) {
  extern __shared__ unsigned char smem_raw[];
  const int np = n + (n & 1), half = np / 2;
  z64* Vs = reinterpret_cast<z64*>(smem_raw);          // rows_per_wg x n, element (r, c) at c * rows + r
  Rot* rs = reinterpret_cast<Rot*>(Vs + rows_per_wg * n);  // kRing x half
  const int bt = blockIdx.y;
  const Rot* log = logb + bt * slog;
  z64* V = Vb + bt * sV;
  const int r0 = blockIdx.x * rows_per_wg;
  const int rows = min(rows_per_wg, n - r0);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < rows * n; e += nt) {
    const int r = e % rows, c = e / rows;
    Vs[c * rows + r] = mk<double>((r0 + r) == c ? 1.0 : 0.0, 0.0);
  }
  const int nr = nrounds[bt];
  for (int t0 = 0; t0 < nr; t0 += kRing) {
    const int cnt = min(kRing, nr - t0);
    __syncthreads();
    for (int e = tid; e < cnt * half; e += nt) rs[e] = log[(int64_t)t0 * half + e];
    __syncthreads();
    for (int u = 0; u < cnt; ++u) {
      const int rr = (t0 + u) % (np - 1);
      for (int e = tid; e < rows * half; e += nt) {
        const int r = e % rows, k = e / rows;
        int a = rr_slot(k, rr, np), b = rr_slot(np - 1 - k, rr, np);
        if (a > b) { const int tmp = a; a = b; b = tmp; }
        if (b >= n) continue;
        const Rot R = rs[u * half + k];
        const z64 v0 = Vs[a * rows + r], v1 = Vs[b * rows + r];
        const z64 v1e = cmul<double>(v1, R.e);
        Vs[a * rows + r] = cadd<double>(cscale<double>(v0, R.c), cscale<double>(v1e, -R.s));
        Vs[b * rows + r] = cadd<double>(cscale<double>(v0, R.s), cscale<double>(v1e, R.c));
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < rows * n; e += nt) {
    const int r = e % rows, c = e / rows;
    V[(r0 + r) + (int64_t)c * ldv] = Vs[c * rows + r];
  }
}

constexpr int kJacobiMaxSweeps = 40;

bool heev_lds(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V,
              int64_t ldv, int64_t sV, int batch, DevMem& logbuf) {
  if (n > 128 || n < 1) return false;
  const int np = n + (n & 1), half = np / 2;
  const int max_rounds = kJacobiMaxSweeps * (np - 1);
  const int64_t slog = (int64_t)max_rounds * half;
  logbuf.ensure(sizeof(Rot) * slog * batch + sizeof(int) * (batch + 4) + 64);
  Rot* log = logbuf.as<Rot>();
  int* nr = reinterpret_cast<int*>(log + slog * batch);
  const int nblk = half * (half + 1) / 2;
  const size_t lds = sizeof(z64) * (size_t)n * (n + 1) / 2 + sizeof(Rot) * kRing * half + 2 * sizeof(int) * half +
                     2 * sizeof(unsigned short) * nblk + 64;
  HIPCK(hipFuncSetAttribute((const void*)k_jacobi_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_jacobi_lds, dim3(batch), dim3(n <= 32 ? 256 : 1024), lds, st, n, A, lda, sA, w, sw, log, slog,
                     max_rounds, nr);
  HIPCK(hipGetLastError());
  const int rows = n <= 32 ? n : 32;
  const size_t lds2 = sizeof(z64) * (size_t)rows * n + sizeof(Rot) * kRing * half;
  HIPCK(hipFuncSetAttribute((const void*)k_rot_apply, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
  hipLaunchKernelGGL(k_rot_apply, dim3((n + rows - 1) / rows, batch), dim3(256), lds2, st, n, rows, log, slog, nr, V,
                     ldv, sV);
  HIPCK(hipGetLastError());
  return true;
}

// ------------------------------------------------------------------ pivoted Cholesky in LDS
// G (n x n Hermitian PSD, ldg) read-only.  Uinv (n x r, ldu): row perm[k] holds
// row k of L^-H; rank r to *rank.
__global__ void __launch_bounds__(1024) k_pchol_lds(int n, const z64* G, int64_t ldg, double tol, int* rank,
                                                    z64* Uinv, int64_t ldu) {
  extern __shared__ unsigned char smem_raw[];
  z64* P = reinterpret_cast<z64*>(smem_raw);        // packed lower n(n+1)/2
  z64* tmp = P + n * (n + 1) / 2;                   // n
  int* perm = reinterpret_cast<int*>(tmp + n);      // n
  __shared__ double bv[16];
  __shared__ int bi[16];
  __shared__ int rk, piv;
  __shared__ double d0;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    if (i > j) {
      const z64 a = G[i + (int64_t)j * ldg], b = G[j + (int64_t)i * ldg];
      P[pk(i, j)] = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    } else if (i == j) {
      P[pk(i, i)] = mk<double>(G[i + (int64_t)i * ldg].x, 0.0);
    }
  }
  for (int i = tid; i < n; i += nt) perm[i] = i;
  if (tid == 0) rk = n;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // parallel argmax of the trailing diagonal (ties -> smallest index): waves then block
    double best = -1.0;
    int bidx = n;
    for (int i = k + tid; i < n; i += nt) {
      const double v = P[pk(i, i)].x;
      if (v > best) { best = v; bidx = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bidx, o, 64);
      if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
    }
    if ((tid & 63) == 0) {
      bv[tid >> 6] = best;
      bi[tid >> 6] = bidx;
    }
    __syncthreads();
    if (tid == 0) {
      double b0 = bv[0];
      int i0 = bi[0];
      for (int wv = 1; wv < (nt >> 6); ++wv)
        if (bv[wv] > b0 || (bv[wv] == b0 && bi[wv] < i0)) { b0 = bv[wv]; i0 = bi[wv]; }
      if (k == 0) d0 = b0;
      piv = i0;
      if (!(b0 > tol * d0) || !(b0 > 0.0)) rk = k;
    }
    __syncthreads();
    if (rk == k) break;
    const int b = piv;
    if (b != k) {
      // symmetric interchange of k and b (rows of L for columns < k included)
      for (int m = tid; m < n; m += nt) {
        if (m == k || m == b) continue;
        const z64 t1 = pget(P, k, m), t2 = pget(P, b, m);
        pset(P, k, m, t2);
        pset(P, b, m, t1);
      }
      if (tid == 0) {
        const z64 dk = P[pk(k, k)];
        P[pk(k, k)] = P[pk(b, b)];
        P[pk(b, b)] = dk;
        const z64 x = P[pk(b, k)];
        P[pk(b, k)] = mk<double>(x.x, -x.y);
        const int t = perm[k];
        perm[k] = perm[b];
        perm[b] = t;
      }
      __syncthreads();
    }
    const double lkk = sqrt(P[pk(k, k)].x);
    for (int i = k + 1 + tid; i < n; i += nt) P[pk(i, k)] = cscale<double>(P[pk(i, k)], 1.0 / lkk);
    __syncthreads();
    if (tid == 0) P[pk(k, k)] = mk<double>(lkk, 0.0);
    const int m = n - k - 1;
    for (int e = tid; e < m * (m + 1) / 2; e += nt) {
      int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (ii * (ii + 1) / 2 > e) --ii;
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int jj = e - ii * (ii + 1) / 2;
      const int i = k + 1 + ii, j = k + 1 + jj;  // i >= j
      const z64 li = P[pk(i, k)], lj = P[pk(j, k)];
      z64 v = csub<double>(P[pk(i, j)], cmul<double>(li, mk<double>(lj.x, -lj.y)));
      if (i == j) v.y = 0.0;
      P[pk(i, j)] = v;
    }
    __syncthreads();
  }
  const int r = rk;
  // in-place inverse of the r x r lower factor, columns right to left:
  // Linv[j][j] = 1/L[j][j]; Linv[i][j] = -(sum_{m=j+1..i} Linv[i][m] L[m][j]) / L[j][j]
  for (int j = r - 1; j >= 0; --j) {
    const double ljj = P[pk(j, j)].x;
    for (int i = j + 1 + tid; i < r; i += nt) {
      double sx = 0, sy = 0;
      for (int m2 = j + 1; m2 <= i; ++m2) {
        const z64 a = P[pk(i, m2)], l = P[pk(m2, j)];
        sx += a.x * l.x - a.y * l.y;
        sy += a.x * l.y + a.y * l.x;
      }
      tmp[i] = mk<double>(-sx / ljj, -sy / ljj);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < r; i += nt) P[pk(i, j)] = tmp[i];
    if (tid == 0) P[pk(j, j)] = mk<double>(1.0 / ljj, 0.0);
    __syncthreads();
  }
  // Uinv[perm[k]][j] = (L^-H)[k][j] = conj(Linv[j][k]) for k <= j < r; zero elsewhere
  for (int e = tid; e < n * r; e += nt) {
    const int row = e % n, j = e / n;
    Uinv[row + (int64_t)j * ldu] = mk<double>(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int k = e % r, j = e / r;
    if (k <= j) {
      const z64 v = P[pk(j, k)];
      Uinv[perm[k] + (int64_t)j * ldu] = mk<double>(v.x, -v.y);
    }
  }
  if (tid == 0) *rank = r;
}

bool pchol_inv_lds(hipStream_t st, int n, const z64* G, int64_t ldg, double tol, int* rank, z64* Uinv, int64_t ldu) {
  if (n > 128 || n < 1) return false;
  const size_t lds = sizeof(z64) * ((size_t)n * (n + 1) / 2 + n) + sizeof(int) * n + 64;
  HIPCK(hipFuncSetAttribute((const void*)k_pchol_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_pchol_lds, dim3(1), dim3(1024), lds, st, n, G, ldg, tol, rank, Uinv, ldu);
  HIPCK(hipGetLastError());
  return true;
}

}  // namespace eahp
