// Static parts of a problem built on the device: the ionic potential on the
// FFT box and the projector matrices; plus small reductions over k-points.
#include <cmath>

#include "devcommon.h"
#include "kernels.h"
#include "setup.h"

namespace eahp {

__device__ __forceinline__ int freq_i(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// V_ion(G) = sum_I -4 pi Z_I exp(-|G|^2 r^2 / 2) / (Omega |G|^2) e^{-i G.R_I};
// G = 0: sum_I 2 pi Z_I r^2 / Omega.
__global__ void k_vion_g(int n1, int n2, int n3, Lat L, int natoms, const double* R, const double* Z, double r,
                         double Omega, z64* box) {
  const int64_t Ng = (int64_t)n1 * n2 * n3;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ng; i += (int64_t)gridDim.x * blockDim.x) {
    const int i3 = (int)(i % n3), i2 = (int)((i / n3) % n2), i1 = (int)(i / ((int64_t)n2 * n3));
    const double m1 = freq_i(i1, n1), m2 = freq_i(i2, n2), m3 = freq_i(i3, n3);
    const double gx = L.B[0] * m1 + L.B[3] * m2 + L.B[6] * m3;
    const double gy = L.B[1] * m1 + L.B[4] * m2 + L.B[7] * m3;
    const double gz = L.B[2] * m1 + L.B[5] * m2 + L.B[8] * m3;
    const double g2 = gx * gx + gy * gy + gz * gz;
    double sx = 0, sy = 0;
    for (int I = 0; I < natoms; ++I) {
      const double f = (i == 0) ? 2.0 * M_PI * Z[I] * r * r / Omega
                                : -4.0 * M_PI * Z[I] * exp(-0.5 * g2 * r * r) / (Omega * g2);
      double sn, cs;
      sincos(gx * R[3 * I] + gy * R[3 * I + 1] + gz * R[3 * I + 2], &sn, &cs);
      sx += f * cs;
      sy -= f * sn;
    }
    box[i] = mk<double>(sx, sy);
  }
}

void launch_vion_g(hipStream_t st, int n1, int n2, int n3, const Lat& L, int natoms, const double* R, const double* Z,
                   double r, double Omega, z64* box) {
  hipLaunchKernelGGL(k_vion_g, dim3(2048), dim3(256), 0, st, n1, n2, n3, L, natoms, R, Z, r, Omega, box);
  HIPCK(hipGetLastError());
}

// beta_I(k+G) = Omega^-1/2 2^(3/2) pi^(3/4) rp^(3/2) exp(-|k+G|^2 rp^2/2) e^{-i(k+G).R_I}
__global__ void k_projectors(int64_t npw, const int* box, int n1, int n2, int n3, Lat L, double kx, double ky,
                             double kz, int natoms, const double* R, double rp, double amp0, z64* P, c32* P32) {
  const int64_t tot = npw * natoms;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e % npw;
    const int I = (int)(e / npw);
    const int b = box[g];
    const int i3 = b % n3, i2 = (b / n3) % n2, i1 = b / (n2 * n3);
    const double m1 = freq_i(i1, n1), m2 = freq_i(i2, n2), m3 = freq_i(i3, n3);
    const double qx = L.B[0] * m1 + L.B[3] * m2 + L.B[6] * m3 + kx;
    const double qy = L.B[1] * m1 + L.B[4] * m2 + L.B[7] * m3 + ky;
    const double qz = L.B[2] * m1 + L.B[5] * m2 + L.B[8] * m3 + kz;
    const double q2 = qx * qx + qy * qy + qz * qz;
    const double amp = amp0 * exp(-0.5 * q2 * rp * rp);
    double sn, cs;
    sincos(qx * R[3 * I] + qy * R[3 * I + 1] + qz * R[3 * I + 2], &sn, &cs);
    const z64 v = mk<double>(amp * cs, -amp * sn);
    P[e] = v;
    P32[e] = mk<float>((float)v.x, (float)v.y);
  }
}

void launch_projectors(hipStream_t st, int64_t npw, const int* box, int n1, int n2, int n3, const Lat& L,
                       const double k[3], int natoms, const double* R, double rp, double Omega, z64* P, c32* P32) {
  if (npw * natoms == 0) return;
  // Omega^-1/2 2^(3/2) pi^(3/4) rp^(3/2)
  const double amp0 = std::pow(Omega, -0.5) * std::pow(2.0, 1.5) * std::pow(M_PI, 0.75) * std::pow(rp, 1.5);
  hipLaunchKernelGGL(k_projectors, dim3(1024), dim3(256), 0, st, npw, box, n1, n2, n3, L, k[0], k[1], k[2], natoms, R,
                     rp, amp0, P, P32);
  HIPCK(hipGetLastError());
}

// out = scale * sum_{k, j} w_k vals[k * p + j]   (single work-group, fixed order)
__global__ void __launch_bounds__(256) k_wsum(int nk, int p, const double* vals, const double* kw, double scale,
                                              double* out) {
  __shared__ double sh[16];
  double s = 0;
  for (int e = threadIdx.x; e < nk * p; e += blockDim.x) s += kw[e / p] * vals[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = scale * s;
}
void weighted_sum(hipStream_t st, int nk, int p, const double* vals, const double* kw, double scale, double* out) {
  hipLaunchKernelGGL(k_wsum, dim3(1), dim3(256), 0, st, nk, p, vals, kw, scale, out);
  HIPCK(hipGetLastError());
}

// out[c] = sum over m blocks of part[b*stride + c] for c < ncomp
__global__ void __launch_bounds__(256) k_sum_strided(int m, int stride, int c, const double* part, double scale,
                                                     double* out) {
  __shared__ double sh[16];
  double s = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += part[i * stride + c];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = scale * s;
}
void sum_strided(hipStream_t st, int m, int stride, int c, const double* part, double scale, double* out) {
  hipLaunchKernelGGL(k_sum_strided, dim3(1), dim3(256), 0, st, m, stride, c, part, scale, out);
  HIPCK(hipGetLastError());
}

// Mirror the strictly upper block A[0:q, q:q+r] into A[q:q+r, 0:q] (conjugate transpose)
// and Hermitise the diagonal block A[q:q+r, q:q+r].
__global__ void k_border_mirror(int q, int r, z64* A, int64_t lda) {
  const int tot = (q + r) * r;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int i = e % (q + r), j = e / (q + r);  // element (i, q + j) of the new block column
    if (i < q) {
      const z64 v = A[i + (int64_t)(q + j) * lda];
      A[(q + j) + (int64_t)i * lda] = mk<double>(v.x, -v.y);
    }
  }
}
void border_mirror(hipStream_t st, int q, int r, z64* A, int64_t lda) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_border_mirror, dim3(std::min(1024, ((q + r) * r + 255) / 256)), dim3(256), 0, st, q, r, A, lda);
  HIPCK(hipGetLastError());
}

// Copy a rows x cols column-major block (complex128) between leading dimensions.
__global__ void k_copy2d(int rows, int cols, const z64* S, int64_t lds, z64* D, int64_t ldd) {
  const int64_t tot = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % rows), j = (int)(e / rows);
    D[i + j * ldd] = S[i + j * lds];
  }
}
void copy2d(hipStream_t st, int rows, int cols, const z64* S, int64_t lds, z64* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return;
  const int nb = (int)std::min<int64_t>(4096, ((int64_t)rows * cols + 255) / 256);
  hipLaunchKernelGGL(k_copy2d, dim3(nb), dim3(256), 0, st, rows, cols, S, lds, D, ldd);
  HIPCK(hipGetLastError());
}

// min over n doubles (single work-group) -> out
__global__ void __launch_bounds__(256) k_minval(int n, const double* v, double* out) {
  __shared__ double sh[256];
  double m = 1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, v[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}
void minval(hipStream_t st, int n, const double* v, double* out) {
  hipLaunchKernelGGL(k_minval, dim3(1), dim3(256), 0, st, n, v, out);
  HIPCK(hipGetLastError());
}

__global__ void __launch_bounds__(256) k_maxval(int n, const double* v, double* out) {
  __shared__ double sh[256];
  double m = -1e300;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}
void maxval(hipStream_t st, int n, const double* v, double* out) {
  hipLaunchKernelGGL(k_maxval, dim3(1), dim3(256), 0, st, n, v, out);
  HIPCK(hipGetLastError());
}

// two-level minimum over a long array
__global__ void __launch_bounds__(256) k_minpart(int64_t n, const double* v, double* part) {
  __shared__ double sh[256];
  double m = 1e300;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmin(m, v[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
void minval_big(hipStream_t st, int64_t n, const double* v, double* out, DevMem& part) {
  part.ensure(sizeof(double) * 1024);
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256));
  hipLaunchKernelGGL(k_minpart, dim3(nb), dim3(256), 0, st, n, v, part.as<double>());
  hipLaunchKernelGGL(k_minval, dim3(1), dim3(256), 0, st, nb, part.as<double>(), out);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
