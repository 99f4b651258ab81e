// Complex block products and vector reductions for tall-skinny frames.
//
// gemm_hn: C = alpha A^H B + beta C (the outer product V^* W of Sec. 5.1:
//          Gram matrices, Lambda, projector coefficients P^H X).  The row
//          dimension n (plane waves) is split across work-groups; each writes a
//          partial tile and a second kernel sums the partials in a fixed order,
//          so results do not depend on scheduling.
// gemm_nn: C = alpha A M + beta C (frame times small matrix: Phi Lambda, the
//          retraction Psi S^-1, the FOM update V Y, projector expansion P B).
#include "devcommon.h"
#include "kernels.h"

namespace eahp {

constexpr int TB = 64;   // output tile edge
constexpr int KC = 16;   // rows / inner dimension per LDS chunk

// ------------------------------------------------------------------ gemm_hn
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_hn(int64_t n, int a, int b, const cplx<T>* __restrict__ A, int64_t lda,
                                                 const cplx<T>* __restrict__ B, int64_t ldb, int64_t rows_per_split,
                                                 cplx<T>* __restrict__ part, int64_t sA, int64_t sB) {
  __shared__ cplx<T> As[KC][TB + 1];
  __shared__ cplx<T> Bs[KC][TB + 1];
  const int tiles_a = (a + TB - 1) / TB;
  const int ta = blockIdx.x % tiles_a, tb = blockIdx.x / tiles_a;
  const int split = blockIdx.y;
  const int batch = blockIdx.z;
  A += batch * sA;
  B += batch * sB;
  const int64_t r0 = split * rows_per_split;
  const int64_t r1 = min(n, r0 + rows_per_split);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  cplx<T> acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = mk<T>(0, 0);
  const int lr = threadIdx.x & 15;   // row within chunk
  const int lc = threadIdx.x >> 4;   // 0..15 column group
  for (int64_t r = r0; r < r1; r += KC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = lc + 16 * q;
      const int64_t row = r + lr;
      const int ia = ta * TB + col, jb = tb * TB + col;
      As[lr][col] = (row < r1 && ia < a) ? A[row + ia * lda] : mk<T>(0, 0);
      Bs[lr][col] = (row < r1 && jb < b) ? B[row + jb * ldb] : mk<T>(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      cplx<T> av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = As[k][tx + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = Bs[k][ty + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[u][v].x += av[u].x * bv[v].x + av[u].y * bv[v].y;
          acc[u][v].y += av[u].x * bv[v].y - av[u].y * bv[v].x;
        }
    }
    __syncthreads();
  }
  // partial layout: [batch][split][b][a]
  cplx<T>* P = part + ((int64_t)batch * gridDim.y + split) * (int64_t)a * b;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ta * TB + tx + 16 * u, j = tb * TB + ty + 16 * v;
      if (i < a && j < b) P[i + (int64_t)j * a] = acc[u][v];
    }
}

template <typename T>
__global__ void k_gemm_hn_reduce(int a, int b, int nsplit, const cplx<T>* __restrict__ part, cplx<T>* C, int64_t ldc,
                                 double alpha, double beta, int64_t sC) {
  const int batch = blockIdx.y;
  const int64_t ab = (int64_t)a * b;
  const cplx<T>* P = part + (int64_t)batch * nsplit * ab;
  C += batch * sC;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ab; e += (int64_t)gridDim.x * blockDim.x) {
    double sx = 0, sy = 0;
    for (int s = 0; s < nsplit; ++s) {
      const cplx<T> v = P[s * ab + e];
      sx += (double)v.x;
      sy += (double)v.y;
    }
    const int i = (int)(e % a), j = (int)(e / a);
    cplx<T>* c = C + i + j * ldc;
    cplx<T> o;
    if (beta == 0.0) {
      o = mk<T>((T)(alpha * sx), (T)(alpha * sy));
    } else {
      o = mk<T>((T)(alpha * sx + beta * (double)c->x), (T)(alpha * sy + beta * (double)c->y));
    }
    *c = o;
  }
}

template <typename T>
void gemm_hn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B, int64_t ldb,
             cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch, int64_t sA, int64_t sB,
             int64_t sC) {
  if (a <= 0 || b <= 0 || batch <= 0) return;
  const int tiles = ((a + TB - 1) / TB) * ((b + TB - 1) / TB);
  // enough work-groups to fill 256 CUs, chunks of at least 4 KC rows
  int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>((n + 4 * KC - 1) / (4 * KC), (1024 + tiles * batch - 1) / (tiles * batch)));
  int64_t rps = (n + nsplit - 1) / nsplit;
  rps = ((rps + KC - 1) / KC) * KC;
  nsplit = std::max<int64_t>(1, (n + rps - 1) / rps);
  if (n <= 0) { nsplit = 1; rps = 0; }
  part.ensure(sizeof(cplx<T>) * (size_t)nsplit * a * b * batch);
  // with n == 0 the kernel writes zero partials
  hipLaunchKernelGGL((k_gemm_hn<T>), dim3(tiles, (unsigned)nsplit, batch), dim3(256), 0, st, n, a, b, A, lda, B, ldb,
                     rps, part.as<cplx<T>>(), sA, sB);
  HIPCK(hipGetLastError());
  const int64_t ab = (int64_t)a * b;
  const int nb = (int)std::min<int64_t>(1024, (ab + 255) / 256);
  hipLaunchKernelGGL((k_gemm_hn_reduce<T>), dim3(nb, batch), dim3(256), 0, st, a, b, (int)nsplit,
                     part.as<cplx<T>>(), C, ldc, alpha, beta, sC);
  HIPCK(hipGetLastError());
}

// ------------------------------------------------------------------ gemm_nn
template <typename T>
__global__ void __launch_bounds__(256) k_gemm_nn(int64_t n, int a, int b, const cplx<T>* __restrict__ A, int64_t lda,
                                                 const cplx<T>* __restrict__ M, int64_t ldm, int opM,
                                                 cplx<T>* __restrict__ C, int64_t ldc, double are, double aim,
                                                 double beta, int64_t sA, int64_t sM, int64_t sC) {
  __shared__ cplx<T> As[KC][TB + 1];  // [k][row]
  __shared__ cplx<T> Ms[KC][TB + 1];  // [k][col]
  const int batch = blockIdx.z;
  A += batch * sA;
  M += batch * sM;
  C += batch * sC;
  const int64_t row0 = (int64_t)blockIdx.x * TB;
  const int col0 = blockIdx.y * TB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  cplx<T> acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = mk<T>(0, 0);
  for (int k0 = 0; k0 < a; k0 += KC) {
    // A chunk: 64 rows x KC columns; consecutive threads take consecutive rows
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;  // 0..1023
      const int rr = e & 63, kk = e >> 6;   // kk 0..15
      const int64_t row = row0 + rr;
      As[kk][rr] = (row < n && k0 + kk < a) ? A[row + (int64_t)(k0 + kk) * lda] : mk<T>(0, 0);
      const int cc = e & 63, mk_ = e >> 6;
      const int j = col0 + cc, kidx = k0 + mk_;
      cplx<T> mv = mk<T>(0, 0);
      if (j < b && kidx < a) {
        if (opM == 0) mv = M[kidx + (int64_t)j * ldm];
        else {
          const cplx<T> t = M[j + (int64_t)kidx * ldm];
          mv = mk<T>(t.x, -t.y);
        }
      }
      Ms[mk_][cc] = mv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      cplx<T> av[4], mv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = As[k][tx + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) mv[v] = Ms[k][ty + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[u][v].x += av[u].x * mv[v].x - av[u].y * mv[v].y;
          acc[u][v].y += av[u].x * mv[v].y + av[u].y * mv[v].x;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = row0 + tx + 16 * u;
      const int j = col0 + ty + 16 * v;
      if (i < n && j < b) {
        cplx<T>* c = C + i + (int64_t)j * ldc;
        const double x = acc[u][v].x, y = acc[u][v].y;
        double ox = are * x - aim * y, oy = are * y + aim * x;
        if (beta != 0.0) {
          ox += beta * (double)c->x;
          oy += beta * (double)c->y;
        }
        *c = mk<T>((T)ox, (T)oy);
      }
    }
}

template <typename T>
void gemm_nn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M, int64_t ldm,
             int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta, int batch, int64_t sA,
             int64_t sM, int64_t sC) {
  if (n <= 0 || b <= 0 || batch <= 0) return;
  dim3 grid((unsigned)((n + TB - 1) / TB), (b + TB - 1) / TB, batch);
  hipLaunchKernelGGL((k_gemm_nn<T>), grid, dim3(256), 0, st, n, a, b, A, lda, M, ldm, opM, C, ldc, alpha_re, alpha_im,
                     beta, sA, sM, sC);
  HIPCK(hipGetLastError());
}

template void gemm_hn<double>(hipStream_t, int64_t, int, int, const z64*, int64_t, const z64*, int64_t, z64*, int64_t,
                              double, double, DevMem&, int, int64_t, int64_t, int64_t);
template void gemm_hn<float>(hipStream_t, int64_t, int, int, const c32*, int64_t, const c32*, int64_t, c32*, int64_t,
                             double, double, DevMem&, int, int64_t, int64_t, int64_t);
template void gemm_nn<double>(hipStream_t, int64_t, int, int, const z64*, int64_t, const z64*, int64_t, int, z64*,
                              int64_t, double, double, double, int, int64_t, int64_t, int64_t);
template void gemm_nn<float>(hipStream_t, int64_t, int, int, const c32*, int64_t, const c32*, int64_t, int, c32*,
                             int64_t, double, double, double, int, int64_t, int64_t, int64_t);

// ------------------------------------------------------------------ vectors
template <typename T>
__global__ void k_axpby(int64_t n, double a, const cplx<T>* x, double b, cplx<T>* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const cplx<T> xv = x[i];
    const cplx<T> yv = y[i];
    y[i] = (b == 0.0) ? mk<T>((T)(a * xv.x), (T)(a * xv.y)) : mk<T>((T)(a * xv.x + b * yv.x), (T)(a * xv.y + b * yv.y));
  }
}
template <typename T>
void axpby(hipStream_t st, int64_t n, double a, const cplx<T>* x, double b, cplx<T>* y) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL((k_axpby<T>), dim3(nb), dim3(256), 0, st, n, a, x, b, y);
  HIPCK(hipGetLastError());
}
template void axpby<double>(hipStream_t, int64_t, double, const z64*, double, z64*);
template void axpby<float>(hipStream_t, int64_t, double, const c32*, double, c32*);

constexpr int kRedBlocks = 1024;

template <typename C>
__global__ void __launch_bounds__(256) k_dot_re(int64_t n, const C* x, const C* y, double* part) {
  __shared__ double sh[16];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const C a = x[i], b = y[i];
    s += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void __launch_bounds__(256) k_sum_partials(int m, const double* part, double* out) {
  __shared__ double sh[16];
  double s = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}
template <typename C>
static void dot_re_impl(hipStream_t st, int64_t n, const C* x, const C* y, double* out_dev, DevMem& part) {
  part.ensure(sizeof(double) * kRedBlocks);
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + 255) / 256));
  hipLaunchKernelGGL((k_dot_re<C>), dim3(nb), dim3(256), 0, st, n, x, y, part.as<double>());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, nb, part.as<double>(), out_dev);
  HIPCK(hipGetLastError());
}
void dot_re(hipStream_t st, int64_t n, const z64* x, const z64* y, double* out_dev, DevMem& part) {
  dot_re_impl(st, n, x, y, out_dev, part);
}
void dot_re(hipStream_t st, int64_t n, const c32* x, const c32* y, double* out_dev, DevMem& part) {
  dot_re_impl(st, n, x, y, out_dev, part);
}

// out[j] = sum_i w_i |X_ij|^2 (w == nullptr: w_i = 1); one work-group per column
__global__ void __launch_bounds__(256) k_col_wnorm2(int64_t n, const z64* X, int64_t ldx, const double* w, double* out) {
  __shared__ double sh[16];
  const z64* x = X + blockIdx.x * ldx;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const z64 v = x[i];
    s += (w ? w[i] : 1.0) * (v.x * v.x + v.y * v.y);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}
void col_weighted_norm2(hipStream_t st, int64_t n, int ncols, const z64* X, int64_t ldx, const double* w, double* out) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_col_wnorm2, dim3(ncols), dim3(256), 0, st, n, X, ldx, w, out);
  HIPCK(hipGetLastError());
}

template <typename S, typename D>
__global__ void k_convert(int64_t n, const S* src, D* dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    dst[i].x = src[i].x;
    dst[i].y = src[i].y;
  }
}
template <typename T>
void convert(hipStream_t st, int64_t n, const void* src, int src_fp64, void* dst, int dst_fp64) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (src_fp64 && !dst_fp64)
    hipLaunchKernelGGL((k_convert<z64, c32>), dim3(nb), dim3(256), 0, st, n, (const z64*)src, (c32*)dst);
  else if (!src_fp64 && dst_fp64)
    hipLaunchKernelGGL((k_convert<c32, z64>), dim3(nb), dim3(256), 0, st, n, (const c32*)src, (z64*)dst);
  else if (src_fp64)
    hipLaunchKernelGGL((k_convert<z64, z64>), dim3(nb), dim3(256), 0, st, n, (const z64*)src, (z64*)dst);
  else
    hipLaunchKernelGGL((k_convert<c32, c32>), dim3(nb), dim3(256), 0, st, n, (const c32*)src, (c32*)dst);
  HIPCK(hipGetLastError());
}
template void convert<double>(hipStream_t, int64_t, const void*, int, void*, int);

// D[rows x cols, ldd] = S[rows x cols, lds] with a change of precision
template <typename S, typename D>
__global__ void k_convert2d(int rows, int cols, const S* src, int64_t lds, D* dst, int64_t ldd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    const S v = src[i + j * lds];
    dst[i + j * ldd].x = v.x;
    dst[i + j * ldd].y = v.y;
  }
}
void convert2d(hipStream_t st, int rows, int cols, const c32* src, int64_t lds, z64* dst, int64_t ldd) {
  if ((int64_t)rows * cols <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, ((int64_t)rows * cols + 255) / 256);
  hipLaunchKernelGGL((k_convert2d<c32, z64>), dim3(nb), dim3(256), 0, st, rows, cols, src, lds, dst, ldd);
  HIPCK(hipGetLastError());
}
void convert2d(hipStream_t st, int rows, int cols, const z64* src, int64_t lds, c32* dst, int64_t ldd) {
  if ((int64_t)rows * cols <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, ((int64_t)rows * cols + 255) / 256);
  hipLaunchKernelGGL((k_convert2d<z64, c32>), dim3(nb), dim3(256), 0, st, rows, cols, src, lds, dst, ldd);
  HIPCK(hipGetLastError());
}

// y += a x with x single precision and y double (n complex values)
__global__ void k_axpy_mixed(int64_t n, double a, const c32* x, z64* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const c32 v = x[i];
    y[i].x += a * (double)v.x;
    y[i].y += a * (double)v.y;
  }
}
void axpy_mixed(hipStream_t st, int64_t n, double a, const c32* x, z64* y) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_axpy_mixed, dim3(nb), dim3(256), 0, st, n, a, x, y);
  HIPCK(hipGetLastError());
}

template <typename T>
__global__ void k_tpa(int64_t n, int ncols, const double* kin, const double* alpha, const cplx<T>* X, int64_t ldx,
                      cplx<T>* Y, int64_t ldy) {
  const int j = blockIdx.y;
  const double al = alpha[j];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double f = 1.0 / (kin[i] + al);
    const cplx<T> v = X[i + j * ldx];
    Y[i + j * ldy] = mk<T>((T)(v.x * f), (T)(v.y * f));
  }
}
template <typename T>
void tpa_apply(hipStream_t st, int64_t n, int ncols, const double* kin, const double* alpha, const cplx<T>* X,
               int64_t ldx, cplx<T>* Y, int64_t ldy) {
  if (ncols <= 0 || n <= 0) return;
  const int nb = (int)std::min<int64_t>(256, (n + 255) / 256);
  hipLaunchKernelGGL((k_tpa<T>), dim3(nb, ncols), dim3(256), 0, st, n, ncols, kin, alpha, X, ldx, Y, ldy);
  HIPCK(hipGetLastError());
}
template void tpa_apply<double>(hipStream_t, int64_t, int, const double*, const double*, const z64*, int64_t, z64*,
                                int64_t);
template void tpa_apply<float>(hipStream_t, int64_t, int, const double*, const double*, const c32*, int64_t, c32*,
                               int64_t);

template <typename T>
__global__ void k_scale_rows(int m, int ncols, const double* D, cplx<T>* B, int64_t ldb) {
  const int64_t tot = (int64_t)m * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    cplx<T>* v = B + i + j * ldb;
    const T d = (T)D[i];
    *v = mk<T>(v->x * d, v->y * d);
  }
}
template <typename T>
void scale_rows(hipStream_t st, int m, int ncols, const double* D, cplx<T>* B, int64_t ldb) {
  if (m <= 0 || ncols <= 0) return;
  const int nb = (int)std::min<int64_t>(1024, ((int64_t)m * ncols + 255) / 256);
  hipLaunchKernelGGL((k_scale_rows<T>), dim3(nb), dim3(256), 0, st, m, ncols, D, B, ldb);
  HIPCK(hipGetLastError());
}
template void scale_rows<double>(hipStream_t, int, int, const double*, z64*, int64_t);
template void scale_rows<float>(hipStream_t, int, int, const double*, c32*, int64_t);

}  // namespace eahp
