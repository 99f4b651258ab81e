// Complex block products and vector reductions for tall-skinny frames.
//
// gemm_hn: C = alpha A^H B + beta C (the outer product V^* W of Sec. 5.1:
//          Gram matrices, Lambda, projector coefficients P^H X), deterministic
//          split over the row dimension.
// gemm_nn: C = alpha A M + beta C (frame times small matrix: Phi Lambda, the
//          retraction Psi S^-1, the FOM update V Y, projector expansion P B).
#include "devcommon.h"
#include "kernels.h"
#include "ops.h"

namespace eahp {

template <typename T>
void gemm_hn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                  int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch,
                  int64_t sA, int64_t sB, int64_t sC);
template <typename T>
void gemm_nn_mfma(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M,
                  int64_t ldm, int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta,
                  int batch, int64_t sA, int64_t sM, int64_t sC);

template <typename T>
void gemm_hn_ragged_mfma(hipStream_t st, const Ragged& rg, int64_t nmax, int a, int b, const cplx<T>* A,
                         const cplx<T>* B, int64_t ldb, int64_t sB, cplx<T>* C, int64_t ldc, int64_t sC, double alpha,
                         double beta, DevMem& part, int batch);
template <typename T>
void gemm_nn_ragged_mfma(hipStream_t st, const Ragged& rg, int64_t nmax, int a, int b, const cplx<T>* A,
                         const cplx<T>* M, int64_t ldm, int64_t sM, int opM, cplx<T>* C, int64_t ldc, int64_t sC,
                         double alpha, double beta, int batch);

// Both products run on the matrix cores (gemm_mfma.hip).
template <typename T>
void gemm_hn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B, int64_t ldb,
             cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch, int64_t sA, int64_t sB,
             int64_t sC) {
  if (a <= 0 || b <= 0 || batch <= 0) return;
  const int slot = kProfGemm + (sizeof(T) == 4 ? 2 : 0) + (n < 1024 ? 4 : 0);
  gemm_prof_begin(st, slot);
  gemm_hn_mfma<T>(st, n, a, b, A, lda, B, ldb, C, ldc, alpha, beta, part, batch, sA, sB, sC);
  gemm_prof_end(st, slot, 8.0 * (double)n * a * b * batch);
}

template <typename T>
void gemm_nn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M, int64_t ldm,
             int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta, int batch, int64_t sA,
             int64_t sM, int64_t sC) {
  if (n <= 0 || b <= 0 || batch <= 0) return;
  const int slot = kProfGemm + 1 + (sizeof(T) == 4 ? 2 : 0) + (n < 1024 ? 4 : 0);
  gemm_prof_begin(st, slot);
  gemm_nn_mfma<T>(st, n, a, b, A, lda, M, ldm, opM, C, ldc, alpha_re, alpha_im, beta, batch, sA, sM, sC);
  gemm_prof_end(st, slot, 8.0 * (double)n * a * b * batch);
}

template <typename T>
void gemm_hn_ragged(hipStream_t st, const Ragged& rg, int64_t nmax, int64_t ntot, int a, int b, const cplx<T>* A,
                    const cplx<T>* B, int64_t ldb, int64_t sB, cplx<T>* C, int64_t ldc, int64_t sC, double alpha,
                    double beta, DevMem& part, int batch) {
  if (a <= 0 || b <= 0 || batch <= 0) return;
  const int slot = kProfGemm + (sizeof(T) == 4 ? 2 : 0) + (nmax < 1024 ? 4 : 0);
  gemm_prof_begin(st, slot);
  gemm_hn_ragged_mfma<T>(st, rg, nmax, a, b, A, B, ldb, sB, C, ldc, sC, alpha, beta, part, batch);
  gemm_prof_end(st, slot, 8.0 * (double)ntot * a * b);
}

template <typename T>
void gemm_nn_ragged(hipStream_t st, const Ragged& rg, int64_t nmax, int64_t ntot, int a, int b, const cplx<T>* A,
                    const cplx<T>* M, int64_t ldm, int64_t sM, int opM, cplx<T>* C, int64_t ldc, int64_t sC,
                    double alpha, double beta, int batch) {
  if (nmax <= 0 || b <= 0 || batch <= 0) return;
  const int slot = kProfGemm + 1 + (sizeof(T) == 4 ? 2 : 0) + (nmax < 1024 ? 4 : 0);
  gemm_prof_begin(st, slot);
  gemm_nn_ragged_mfma<T>(st, rg, nmax, a, b, A, M, ldm, sM, opM, C, ldc, sC, alpha, beta, batch);
  gemm_prof_end(st, slot, 8.0 * (double)ntot * a * b);
}

template void gemm_hn_ragged<double>(hipStream_t, const Ragged&, int64_t, int64_t, int, int, const z64*, const z64*,
                                     int64_t, int64_t, z64*, int64_t, int64_t, double, double, DevMem&, int);
template void gemm_hn_ragged<float>(hipStream_t, const Ragged&, int64_t, int64_t, int, int, const c32*, const c32*,
                                    int64_t, int64_t, c32*, int64_t, int64_t, double, double, DevMem&, int);
template void gemm_nn_ragged<double>(hipStream_t, const Ragged&, int64_t, int64_t, int, int, const z64*, const z64*,
                                     int64_t, int64_t, int, z64*, int64_t, int64_t, double, double, int);
template void gemm_nn_ragged<float>(hipStream_t, const Ragged&, int64_t, int64_t, int, int, const c32*, const c32*,
                                    int64_t, int64_t, int, c32*, int64_t, int64_t, double, double, int);

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

// The same over the k-blocks of a stacked frame of p columns, one launch:
// out[k p + j] over the npw_k rows of block k, weights |k+G|^2/2 (kin) or 1
__global__ void __launch_bounds__(256) k_frame_wnorm2(const KDesc* __restrict__ kd, int p, const z64* X, int kin,
                                                      double* out) {
  __shared__ double sh[16];
  const int j = blockIdx.x, k = blockIdx.y;
  const int64_t n = kd[k].npw;
  const z64* x = X + p * kd[k].off + (int64_t)j * n;
  const double* w = kin ? kd[k].kin : nullptr;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const z64 v = x[i];
    s += (w ? w[i] : 1.0) * (v.x * v.x + v.y * v.y);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[(int64_t)k * p + j] = s;
}
void frame_col_wnorm2(hipStream_t st, const KDesc* kd, int nk, int p, const z64* X, int kin, double* out) {
  if (nk <= 0 || p <= 0) return;
  hipLaunchKernelGGL(k_frame_wnorm2, dim3(p, nk), dim3(256), 0, st, kd, p, X, kin, out);
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
