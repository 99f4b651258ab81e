// Kohn-Sham H-apply, density and potentials on gfx950.
//
// Local potential (Sec. 5.1; plane-wave discretisation): for each orbital the
// sphere coefficients are scattered into a pruned FFT box, transformed to the
// grid, multiplied by V_eff and transformed back.  The box is never
// materialised: only the x-planes that hold plane waves ("active planes") are
// kept, in an intermediate buffer T laid out [column][plane s][i2][i3].
//
//   inv_yz  : one work-group per (plane, column); scatter the plane's sphere
//             coefficients into a whole i2 x i3 plane in LDS, inverse z- and
//             y-transforms in LDS, one coalesced store of the plane.
//   x_local : one work-group per tile of (i2, i3) positions and a chunk of
//             columns; loads the active-plane values of the tile, inverse
//             x-transform, multiply by V_eff (tile kept in LDS and reused by
//             the chunk's columns), forward x-transform, stores the active
//             planes back.
//   fwd_yz  : forward y- and z-transforms of a plane in LDS, gather of the
//             sphere coefficients, scaled by 1/N_g, plus the kinetic term.
//   x_density: inverse x-transform of every column of a tile and accumulation
//             of w_k f |psi|^2 / Omega in registers (fixed order, no atomics).
#include <algorithm>
#include <cmath>

#include "devcommon.h"
#include "kernels.h"
#include "regfft.h"

// line lengths with register transforms (x lines, square yz planes), as (n1, N1, N2)
#define EAHP_XREG_SIZES(X)                                                                                     \
  X(12, 3, 4) X(15, 3, 5) X(16, 4, 4) X(18, 3, 6) X(20, 4, 5) X(24, 4, 6) X(27, 3, 9) X(30, 5, 6) X(32, 4, 8) X(36, 6, 6) X(40, 5, 8) X(45, 5, 9)   \
  X(48, 6, 8) X(50, 5, 10) X(54, 6, 9) X(60, 6, 10) X(64, 8, 8) X(72, 8, 9) X(75, 5, 15) X(80, 8, 10)          \
  X(81, 9, 9) X(90, 9, 10) X(96, 8, 12) X(100, 10, 10) X(108, 9, 12) X(120, 10, 12) X(128, 8, 16) X(144, 12, 12)
// square yz planes whose padded plane fits LDS in single precision (double: up to 100)
#define EAHP_YZREG_SIZES(X)                                                                                    \
  X(12, 3, 4) X(15, 3, 5) X(16, 4, 4) X(18, 3, 6) X(20, 4, 5) X(24, 4, 6) X(27, 3, 9) X(30, 5, 6) X(32, 4, 8) X(36, 6, 6) X(40, 5, 8) X(45, 5, 9)   \
  X(48, 6, 8) X(50, 5, 10) X(54, 6, 9) X(60, 6, 10) X(64, 8, 8) X(72, 8, 9) X(75, 5, 15) X(80, 8, 10)          \
  X(81, 9, 9) X(90, 9, 10) X(96, 8, 12) X(100, 10, 10) X(108, 9, 12) X(120, 10, 12) X(128, 8, 16)


namespace eahp {

template <typename T> __device__ __forceinline__ const T* kin_of(const KDesc& k);
template <> __device__ __forceinline__ const double* kin_of<double>(const KDesc& k) { return k.kin; }
template <> __device__ __forceinline__ const float* kin_of<float>(const KDesc& k) { return k.kin32; }

__device__ __forceinline__ const KDesc& col_kd(const ColMap& cm, int c, int64_t& base) {
  const int slot = c / cm.cpk;
  const int j = c - slot * cm.cpk;
  if (cm.frame == 2) {
    const int kk = cm.kmap[slot];
    base = (int64_t)kk * cm.kstride + (int64_t)j * cm.ld;
    return cm.kd[kk];
  }
  const KDesc& k = cm.kd[cm.k0 + slot];
  base = (cm.frame ? (int64_t)cm.cpk * k.off : 0) + (int64_t)j * k.npw;
  return k;
}

static int pick_maxpts(int64_t pts, int nt) {
  const int64_t per = (pts + nt - 1) / nt;
  if (per <= 4) return 4;
  if (per <= 8) return 8;
  if (per <= 16) return 16;
  if (per <= 32) return 32;
  fail(EAHP_EINVAL, "FFT work per thread too large");
}

// ------------------------------------------------------------------ inv_yz
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(1024) k_inv_yz(ColMap cm, GridGeom g, FftPlan pz, FftPlan py,
                                                 const cplx<T>* __restrict__ twz, const cplx<T>* __restrict__ twy,
                                                 const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Tb) {
  extern __shared__ unsigned char smem_raw[];
  const int np = g.n2 * g.n3;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tz = pl + np;
  cplx<T>* ty = tz + g.n3;
  const int s = blockIdx.x, c = blockIdx.y;
  int64_t base;
  const KDesc& k = col_kd(cm, c, base);
  for (int i = threadIdx.x; i < np; i += blockDim.x) pl[i] = mk<T>(0, 0);
  for (int i = threadIdx.x; i < g.n3; i += blockDim.x) tz[i] = twz[i];
  for (int i = threadIdx.x; i < g.n2; i += blockDim.x) ty[i] = twy[i];
  __syncthreads();
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  const cplx<T>* x = X + base;
  const int pbase = g.plane_i1[s] * np;  // box index of the plane start
  for (int r = g0 + threadIdx.x; r < g1; r += blockDim.x) pl[k.box[r] - pbase] = x[r];
  __syncthreads();
  // z-lines only on the rows i2 = m2 mod n2 with |m2| <= m2max (the others are zero)
  lds_fft<T, MAXPTS>(pl, Lines{g.n3, 1, 2 * g.m2max + 1, g.n3, 0, g.n2 - g.m2max, g.n2}, pz, tz, (T)1);
  lds_fft<T, MAXPTS>(pl, Lines{g.n2, g.n3, g.n3, 1, 1}, py, ty, (T)1);
  cplx<T>* out = Tb + ((int64_t)c * g.ns + s) * g.ps;
  for (int i = threadIdx.x; i < np; i += blockDim.x) out[i] = pl[i];
}

// ------------------------------------------------------------------ fwd_yz
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(1024) k_fwd_yz(ColMap cm, GridGeom g, FftPlan pz, FftPlan py,
                                                 const cplx<T>* __restrict__ twz, const cplx<T>* __restrict__ twy,
                                                 const cplx<T>* __restrict__ Tb, const cplx<T>* __restrict__ X,
                                                 cplx<T>* __restrict__ HX, T scale) {
  extern __shared__ unsigned char smem_raw[];
  const int np = g.n2 * g.n3;
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tz = pl + np;
  cplx<T>* ty = tz + g.n3;
  const int s = blockIdx.x, c = blockIdx.y;
  int64_t base;
  const KDesc& k = col_kd(cm, c, base);
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  if (g1 == g0) return;  // block-uniform: this k-point has no plane waves here
  const int pbase = g.plane_i1[s] * np;
  const cplx<T>* in = Tb + ((int64_t)c * g.ns + s) * g.ps;
  for (int i = threadIdx.x; i < np; i += blockDim.x) pl[i] = in[i];
  for (int i = threadIdx.x; i < g.n3; i += blockDim.x) tz[i] = twz[i];
  for (int i = threadIdx.x; i < g.n2; i += blockDim.x) ty[i] = twy[i];
  __syncthreads();
  lds_fft<T, MAXPTS>(pl, Lines{g.n2, g.n3, g.n3, 1, 1}, py, ty, (T)-1);
  // z-lines only where the sphere is gathered: rows with |m2| <= m2max
  lds_fft<T, MAXPTS>(pl, Lines{g.n3, 1, 2 * g.m2max + 1, g.n3, 0, g.n2 - g.m2max, g.n2}, pz, tz, (T)-1);
  const T* kin = kin_of<T>(k);
  const cplx<T>* x = X + base;
  cplx<T>* y = HX + base;
  for (int r = g0 + threadIdx.x; r < g1; r += blockDim.x) {
    const cplx<T> v = pl[k.box[r] - pbase];
    const cplx<T> xv = x[r];
    const T kr = kin[r];
    y[r] = mk<T>(v.x * scale + kr * xv.x, v.y * scale + kr * xv.y);
  }
}

// ------------------------------------------------------------------ x_local
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(512) k_x_local(int ncols, int cb, GridGeom g, int tile, FftPlan px,
                                                 const cplx<T>* __restrict__ twx, const T* __restrict__ V,
                                                 cplx<T>* __restrict__ Tb) {
  extern __shared__ unsigned char smem_raw[];
  const int n1 = g.n1, np = g.n2 * g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);      // n1 x tile, element (i1, t) at i1 * tile + t
  T* vt = reinterpret_cast<T*>(buf + n1 * tile);             // n1 x tile
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(vt + n1 * tile);  // n1
  const int t0 = blockIdx.x * tile;
  const int cnt = min(tile, np - t0);
  const FDiv fc = fdiv_make(cnt), ft = fdiv_make(tile);
  for (int i = threadIdx.x; i < n1; i += blockDim.x) tw[i] = twx[i];
  for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) {
    const int i1 = fdiv_q(e, ft), t = e - i1 * tile;
    vt[e] = t < cnt ? V[(int64_t)i1 * np + t0 + t] : (T)0;
  }
  const int c0 = blockIdx.y * cb;
  const int c1 = min(ncols, c0 + cb);
  const Lines L{n1, tile, tile, 1, 1};
  for (int c = c0; c < c1; ++c) {
    for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) buf[e] = mk<T>(0, 0);
    __syncthreads();
    const cplx<T>* in = Tb + (int64_t)c * g.ns * g.ps + t0;
    for (int e = threadIdx.x; e < g.ns * cnt; e += blockDim.x) {
      const int s = fdiv_q(e, fc), t = e - s * cnt;
      buf[g.plane_i1[s] * tile + t] = in[(int64_t)s * g.ps + t];
    }
    __syncthreads();
    lds_fft<T, MAXPTS>(buf, L, px, tw, (T)1);
    for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) buf[e] = cscale<T>(buf[e], vt[e]);
    __syncthreads();
    lds_fft<T, MAXPTS>(buf, L, px, tw, (T)-1);
    cplx<T>* out = Tb + (int64_t)c * g.ns * g.ps + t0;
    for (int e = threadIdx.x; e < g.ns * cnt; e += blockDim.x) {
      const int s = fdiv_q(e, fc), t = e - s * cnt;
      out[(int64_t)s * g.ps + t] = buf[g.plane_i1[s] * tile + t];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ x_density
template <int MAXPTS>
__global__ void __launch_bounds__(512) k_x_density(ColMap cm, int ncols, int cpg, GridGeom g, int tile, FftPlan px,
                                                   const z64* __restrict__ twx, const z64* __restrict__ Tb,
                                                   double occ_over_omega, double* __restrict__ rho, int accumulate,
                                                   int64_t sgrp) {
  extern __shared__ unsigned char smem_raw[];
  const int n1 = g.n1, np = g.n2 * g.n3;
  z64* buf = reinterpret_cast<z64*>(smem_raw);
  z64* tw = buf + n1 * tile;
  const int t0 = blockIdx.x * tile;
  const int cnt = min(tile, np - t0);
  const FDiv fc = fdiv_make(cnt), ft = fdiv_make(tile);
  for (int i = threadIdx.x; i < n1; i += blockDim.x) tw[i] = twx[i];
  double acc[MAXPTS];
#pragma unroll
  for (int r = 0; r < MAXPTS; ++r) acc[r] = 0.0;
  const Lines L{n1, tile, tile, 1, 1};
  // column group blockIdx.y writes its own partial density (rho + blockIdx.y * sgrp)
  const int cbeg = blockIdx.y * cpg, cend = min(ncols, cbeg + cpg);
  rho += blockIdx.y * sgrp;
  for (int c = cbeg; c < cend; ++c) {
    int64_t base;
    const KDesc& k = col_kd(cm, c, base);
    const double wgt = k.w * occ_over_omega;
    for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) buf[e] = mk<double>(0, 0);
    __syncthreads();
    const z64* in = Tb + (int64_t)c * g.ns * g.ps + t0;
    for (int e = threadIdx.x; e < g.ns * cnt; e += blockDim.x) {
      const int s = fdiv_q(e, fc), t = e - s * cnt;
      buf[g.plane_i1[s] * tile + t] = in[(int64_t)s * g.ps + t];
    }
    __syncthreads();
    lds_fft<double, MAXPTS>(buf, L, px, tw, 1.0);
#pragma unroll
    for (int r = 0; r < MAXPTS; ++r) {
      const int e = threadIdx.x + r * blockDim.x;
      if (e < n1 * tile) {
        const z64 v = buf[e];
        acc[r] += wgt * (v.x * v.x + v.y * v.y);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < MAXPTS; ++r) {
    const int e = threadIdx.x + r * blockDim.x;
    if (e < n1 * tile) {
      const int i1 = fdiv_q(e, ft), t = e - i1 * tile;
      if (t < cnt) {
        double* d = rho + (int64_t)i1 * np + t0 + t;
        *d = accumulate ? *d + acc[r] : acc[r];
      }
    }
  }
}

// ------------------------------------------------------------------ split planes
// Boxes whose (y, z) plane does not fit in LDS run the plane transforms as
// blocks of lines: the z-lines of a block of i2 values (with the sphere
// scatter / gather) and the y-lines of a block of i3 values, each block in
// LDS, with the slab in global memory in between.

// Blocks of lines of a strided array: plane p at base + p * pstride; line l of
// the plane at l * ls, element j at j * es; block b holds lines
// [b * BL, min(nlines, (b + 1) * BL)).  Grid (blocks, planes).
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(512) k_lines_fft(cplx<T>* __restrict__ base, int64_t pstride, int N, int64_t es,
                                                   int64_t ls, int nlines, int BL, FftPlan P,
                                                   const cplx<T>* __restrict__ tw, T sg) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // BL x N, line-major
  cplx<T>* tws = buf + (size_t)BL * N;
  const int l0 = blockIdx.x * BL, nl = min(BL, nlines - l0);
  cplx<T>* pl = base + (int64_t)blockIdx.y * pstride + (int64_t)l0 * ls;
  for (int i = threadIdx.x; i < N; i += blockDim.x) tws[i] = tw[i];
  // consecutive threads along the unit-stride direction of global memory
  if (es == 1) {
    for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
      const int l = e / N, j = e - l * N;
      buf[l * N + j] = pl[l * ls + j];
    }
  } else {
    for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
      const int j = e / nl, l = e - j * nl;
      buf[l * N + j] = pl[l * ls + j * es];
    }
  }
  __syncthreads();
  lds_fft<T, MAXPTS>(buf, Lines{N, 1, nl, N, 0}, P, tws, sg);
  if (es == 1) {
    for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
      const int l = e / N, j = e - l * N;
      pl[l * ls + j] = buf[l * N + j];
    }
  } else {
    for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
      const int j = e / nl, l = e - j * nl;
      pl[l * ls + j * es] = buf[l * N + j];
    }
  }
}

// Inverse z-transform of a block of z-lines (i2 in [b*BZ, ...)) of plane s of
// column c after scattering the sphere coefficients; grid (blocks, ns, ncols).
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(512) k_inv_z_sphere(ColMap cm, GridGeom g, int BZ, FftPlan pz,
                                                      const cplx<T>* __restrict__ twz, const cplx<T>* __restrict__ X,
                                                      cplx<T>* __restrict__ Tb) {
  extern __shared__ unsigned char smem_raw[];
  const int n3 = g.n3, np = g.n2 * g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // BZ x n3
  cplx<T>* tz = buf + (size_t)BZ * n3;
  const int s = blockIdx.y, c = blockIdx.z;
  const int i2a = blockIdx.x * BZ, nl = min(BZ, g.n2 - i2a);
  int64_t base;
  const KDesc& k = col_kd(cm, c, base);
  for (int e = threadIdx.x; e < nl * n3; e += blockDim.x) buf[e] = mk<T>(0, 0);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tz[i] = twz[i];
  __syncthreads();
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  const int pbase = g.plane_i1[s] * np;
  const FDiv f3 = fdiv_make(n3);
  const cplx<T>* x = X + base;
  for (int r = g0 + threadIdx.x; r < g1; r += blockDim.x) {
    const int q = k.box[r] - pbase;
    const int qi = fdiv_q(q, f3);
    const int i2 = qi - i2a;
    if (i2 >= 0 && i2 < nl) buf[i2 * n3 + (q - qi * n3)] = x[r];
  }
  __syncthreads();
  lds_fft<T, MAXPTS>(buf, Lines{n3, 1, nl, n3, 0}, pz, tz, (T)1);
  cplx<T>* out = Tb + ((int64_t)c * g.ns + s) * g.ps + (int64_t)i2a * n3;
  for (int e = threadIdx.x; e < nl * n3; e += blockDim.x) out[e] = buf[e];
}

// Forward z-transform of a block of z-lines, gather of the sphere
// coefficients of the block, times 1/N_g, plus the kinetic term.
template <typename T, int MAXPTS>
__global__ void __launch_bounds__(512) k_fwd_z_sphere(ColMap cm, GridGeom g, int BZ, FftPlan pz,
                                                      const cplx<T>* __restrict__ twz, const cplx<T>* __restrict__ Tb,
                                                      const cplx<T>* __restrict__ X, cplx<T>* __restrict__ HX,
                                                      T scale) {
  extern __shared__ unsigned char smem_raw[];
  const int n3 = g.n3, np = g.n2 * g.n3;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tz = buf + (size_t)BZ * n3;
  const int s = blockIdx.y, c = blockIdx.z;
  const int i2a = blockIdx.x * BZ, nl = min(BZ, g.n2 - i2a);
  int64_t base;
  const KDesc& k = col_kd(cm, c, base);
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  if (g1 == g0) return;  // block-uniform
  const int pbase = g.plane_i1[s] * np;
  const FDiv f3 = fdiv_make(n3);
  const cplx<T>* in = Tb + ((int64_t)c * g.ns + s) * g.ps + (int64_t)i2a * n3;
  for (int e = threadIdx.x; e < nl * n3; e += blockDim.x) buf[e] = in[e];
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tz[i] = twz[i];
  __syncthreads();
  lds_fft<T, MAXPTS>(buf, Lines{n3, 1, nl, n3, 0}, pz, tz, (T)-1);
  const T* kin = kin_of<T>(k);
  const cplx<T>* x = X + base;
  cplx<T>* y = HX + base;
  for (int r = g0 + threadIdx.x; r < g1; r += blockDim.x) {
    const int q = k.box[r] - pbase;
    const int qi = fdiv_q(q, f3);
    const int i2 = qi - i2a;
    if (i2 >= 0 && i2 < nl) {
      const cplx<T> v = buf[i2 * n3 + (q - qi * n3)];
      const cplx<T> xv = x[r];
      const T kr = kin[r];
      y[r] = mk<T>(v.x * scale + kr * xv.x, v.y * scale + kr * xv.y);
    }
  }
}

// ------------------------------------------------------------------ launchers
template <typename T> static size_t plane_lds(const GridGeom& g) {
  return sizeof(cplx<T>) * ((size_t)g.n2 * g.n3 + g.n2 + g.n3);
}

template <typename T, int M>
static void set_lds(const void* f, size_t bytes) {
  HIPCK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

static constexpr size_t kLdsMax = 160 * 1024;

// line block size for lines of length N within an LDS budget
static int line_block(int N, size_t elem, size_t budget) {
  int bl = 64;
  while (bl > 1 && (size_t)bl * N * elem + N * elem > budget) bl /= 2;
  return bl;
}

template <typename T>
static void launch_lines(hipStream_t st, cplx<T>* base, int64_t pstride, int nplanes, int N, int64_t es, int64_t ls,
                         int nlines, const FftPlan& P, const cplx<T>* tw, T sg) {
  const int BL = line_block(N, sizeof(cplx<T>), 64 * 1024);
  const size_t lds = sizeof(cplx<T>) * ((size_t)BL * N + N);
  const int nt = 256;
  dim3 grid((nlines + BL - 1) / BL, nplanes);
  switch (pick_maxpts((int64_t)BL * N, nt)) {
#define CASE(M)                                                                                                 \
  case M:                                                                                                       \
    set_lds<T, M>((const void*)k_lines_fft<T, M>, lds);                                                        \
    hipLaunchKernelGGL((k_lines_fft<T, M>), grid, dim3(nt), lds, st, base, pstride, N, es, ls, nlines, BL, P, tw, \
                       sg);                                                                                     \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
}


// ------------------------------------------------------------------ yz planes, register transforms
// The plane transforms of k_inv_yz / k_fwd_yz for square planes n2 = n3 =
// n = N1 N2 (the register four-step of k_x_local_reg), one work-group of
// 8 waves per (plane, column), the plane in LDS with row stride n + 1.
// z-lines (rows, only |m2| <= m2max) and y-lines (columns) each take 16
// lines per wave and 4 lane groups; every step works in place on its
// line's LDS positions (step B leaves frequency k1 + N1 k2 of a line at
// position N2 k1 + k2, and the next transform or the gather reads it there),
// so each transform needs only the barrier between its two steps and no
// lane holds more than one sub-DFT.  The y-transform reads (forward) or
// writes (inverse) the slab directly: 16 consecutive i3 of one row per lane
// group.
constexpr int kYzThreads = 512;
// waves per SIMD the register allocation must allow: two work-groups of 8
// waves per CU in FP32 (the LDS holds two FP32 planes up to n = 90)
template <typename T> constexpr int yz_waves_per_simd() { return sizeof(T) == 4 ? 4 : 2; }

__device__ __forceinline__ bool row_active(int r, int n, int m2max) { return r <= m2max || r >= n - m2max; }

// one line of the four-step in LDS: element j of the line at base + j * es.
// Step A for the lane's j2 = grp + 4a: x(N2 j1 + j2) -> z(k1; j2) at k1 N2 + j2.
template <typename T, int N1, int N2, bool kSkipInactive>
__device__ __forceinline__ void yz_step_a(cplx<T>* base, int es, int grp, const cplx<T>* tw, T sg, int n, int m2max) {
  constexpr int JA = (N2 + 3) / 4;
#pragma unroll
  for (int a = 0; a < JA; ++a) {
    const int j2 = grp + 4 * a;
    if (j2 < N2) {
      cplx<T> u[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int r = N2 * j1 + j2;
        u[j1] = (!kSkipInactive || row_active(r, n, m2max)) ? base[r * es] : mk<T>(0, 0);
      }
      RegFft<T, N1>::run(u, sg);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        cplx<T> w = tw[j2 * k1];
        w.y *= -sg;  // the table holds exp(-2 pi i m / n)
        base[(k1 * N2 + j2) * es] = k1 == 0 ? u[0] : cmul<T>(u[k1], w);
      }
    }
  }
}

template <typename T, int N1, int N2>
__global__ void __launch_bounds__(kYzThreads, yz_waves_per_simd<T>()) k_inv_yz_reg(ColMap cm, GridGeom g, const cplx<T>* __restrict__ tws,
                                                           const cplx<T>* __restrict__ X, cplx<T>* __restrict__ Tb) {
  constexpr int n = N1 * N2, LS = n + 1, KB = (N1 + 3) / 4;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* P = reinterpret_cast<cplx<T>*>(smem_raw);  // n rows of LS
  cplx<T>* tw = P + n * LS;
  const int s = blockIdx.x, c = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & 15, grp = lane >> 4;
  const int m2 = g.m2max, nrow = 2 * m2 + 1;
  int64_t xb;
  const KDesc& k = col_kd(cm, c, xb);
  for (int i = threadIdx.x; i < n; i += kYzThreads) tw[i] = tws[i];
  for (int e = threadIdx.x; e < nrow * n; e += kYzThreads) {
    const int l = e / n, i3 = e - l * n;
    int r = n - m2 + l;
    r -= r >= n ? n : 0;
    P[r * LS + i3] = mk<T>(0, 0);
  }
  __syncthreads();
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  const int pbase = g.plane_i1[s] * n * n;
  const cplx<T>* x = X + xb;
  for (int q = g0 + threadIdx.x; q < g1; q += kYzThreads) {
    const int e = k.box[q] - pbase;
    const int i2 = e / n;
    P[i2 * LS + (e - i2 * n)] = x[q];
  }
  __syncthreads();
  // z-lines: rows with |m2| <= m2max.  Step B writes each size-N2 DFT back
  // over the positions it read (frequency k1 + N1 k2 at position N2 k1 + k2),
  // so no lane waits for another before writing; the y-lines read the
  // columns in that order.
  const int zpasses = (nrow + 16 * (kYzThreads / 64) - 1) / (16 * (kYzThreads / 64));
  for (int ps = 0; ps < zpasses; ++ps) {
    const int l = (ps * (kYzThreads / 64) + wave) * 16 + t;
    int r = n - m2 + l;
    r -= r >= n ? n : 0;
    cplx<T>* row = P + r * LS;
    if (l < nrow) yz_step_a<T, N1, N2, false>(row, 1, grp, tw, (T)1, n, m2);
    __syncthreads();
    if (l < nrow) {
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int k1 = grp + 4 * b;
        if (k1 < N1) {
          cplx<T> y[N2];
#pragma unroll
          for (int j2 = 0; j2 < N2; ++j2) y[j2] = row[k1 * N2 + j2];
          RegFft<T, N2>::run(y, (T)1);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) row[k1 * N2 + k2] = y[k2];
        }
      }
    }
  }
  __syncthreads();
  // y-lines: every z-frequency i3 (its column at position N2 (i3 mod N1) +
  // i3 div N1), results straight to the slab, one size-N2 DFT at a time
  cplx<T>* out = Tb + ((int64_t)c * g.ns + s) * g.ps;
  constexpr int ypasses = (n + 16 * (kYzThreads / 64) - 1) / (16 * (kYzThreads / 64));
  for (int ps = 0; ps < ypasses; ++ps) {
    const int i3 = (ps * (kYzThreads / 64) + wave) * 16 + t;
    cplx<T>* col = P + (i3 % N1) * N2 + i3 / N1;
    if (i3 < n) yz_step_a<T, N1, N2, true>(col, LS, grp, tw, (T)1, n, m2);
    __syncthreads();
    if (i3 < n) {
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int k1 = grp + 4 * b;
        if (k1 < N1) {
          cplx<T> y[N2];
#pragma unroll
          for (int j2 = 0; j2 < N2; ++j2) y[j2] = col[(k1 * N2 + j2) * LS];
          RegFft<T, N2>::run(y, (T)1);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) out[(k1 + N1 * k2) * n + i3] = y[k2];
        }
      }
    }
  }
}

template <typename T, int N1, int N2>
__global__ void __launch_bounds__(kYzThreads, yz_waves_per_simd<T>()) k_fwd_yz_reg(ColMap cm, GridGeom g, const cplx<T>* __restrict__ tws,
                                                           const cplx<T>* __restrict__ Tb,
                                                           const cplx<T>* __restrict__ X, cplx<T>* __restrict__ HX,
                                                           T scale) {
  constexpr int n = N1 * N2, LS = n + 1, KB = (N1 + 3) / 4, JA = (N2 + 3) / 4;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* P = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* tw = P + n * LS;
  const int s = blockIdx.x, c = blockIdx.y;
  int64_t xb;
  const KDesc& k = col_kd(cm, c, xb);
  const int g0 = k.plane_start[s], g1 = k.plane_start[s + 1];
  if (g1 == g0) return;  // block-uniform: this k-point has no plane waves here
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = lane & 15, grp = lane >> 4;
  const int m2 = g.m2max, nrow = 2 * m2 + 1;
  for (int i = threadIdx.x; i < n; i += kYzThreads) tw[i] = tws[i];
  __syncthreads();
  // y-lines (forward) from the slab: step A loads of rows N2 j1 + j2
  const cplx<T>* in = Tb + ((int64_t)c * g.ns + s) * g.ps;
  constexpr int ypasses = (n + 16 * (kYzThreads / 64) - 1) / (16 * (kYzThreads / 64));
  for (int ps = 0; ps < ypasses; ++ps) {
    const int i3 = (ps * (kYzThreads / 64) + wave) * 16 + t;
    const bool ok = i3 < n;
    cplx<T> u[JA][N1];
#pragma unroll
    for (int a = 0; a < JA; ++a) {
      const int j2 = grp + 4 * a;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) u[a][j1] = (ok && j2 < N2) ? in[(N2 * j1 + j2) * n + i3] : mk<T>(0, 0);
    }
    if (ok) {
#pragma unroll
      for (int a = 0; a < JA; ++a) {
        const int j2 = grp + 4 * a;
        if (j2 < N2) {
          RegFft<T, N1>::run(u[a], (T)-1);
#pragma unroll
          for (int k1 = 0; k1 < N1; ++k1)
            P[(k1 * N2 + j2) * LS + i3] = k1 == 0 ? u[a][0] : cmul<T>(u[a][k1], tw[j2 * k1]);
        }
      }
    }
    __syncthreads();
    // step B in place: frequency k1 + N1 k2 of the column lands in row N2 k1 + k2
    if (ok) {
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int k1 = grp + 4 * b;
        if (k1 < N1) {
          cplx<T> y[N2];
#pragma unroll
          for (int j2 = 0; j2 < N2; ++j2) y[j2] = P[(k1 * N2 + j2) * LS + i3];
          RegFft<T, N2>::run(y, (T)-1);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) P[(k1 * N2 + k2) * LS + i3] = y[k2];
        }
      }
    }
  }
  __syncthreads();
  // z-lines (forward) on the rows the sphere reaches (y-frequency r in row
  // N2 (r mod N1) + r div N1), step B again in place
  const int zpasses = (nrow + 16 * (kYzThreads / 64) - 1) / (16 * (kYzThreads / 64));
  for (int ps = 0; ps < zpasses; ++ps) {
    const int l = (ps * (kYzThreads / 64) + wave) * 16 + t;
    int r = n - m2 + l;
    r -= r >= n ? n : 0;
    cplx<T>* row = P + ((r % N1) * N2 + r / N1) * LS;
    if (l < nrow) yz_step_a<T, N1, N2, false>(row, 1, grp, tw, (T)-1, n, m2);
    __syncthreads();
    if (l < nrow) {
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int k1 = grp + 4 * b;
        if (k1 < N1) {
          cplx<T> y[N2];
#pragma unroll
          for (int j2 = 0; j2 < N2; ++j2) y[j2] = row[k1 * N2 + j2];
          RegFft<T, N2>::run(y, (T)-1);
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) row[k1 * N2 + k2] = y[k2];
        }
      }
    }
  }
  __syncthreads();
  // gather of the sphere (frequency (i2, i3) at row N2 (i2 mod N1) + i2 div N1,
  // column N2 (i3 mod N1) + i3 div N1), scaled, plus the kinetic term
  const int pbase = g.plane_i1[s] * n * n;
  const T* kin = kin_of<T>(k);
  const cplx<T>* x = X + xb;
  cplx<T>* yv = HX + xb;
  for (int q = g0 + threadIdx.x; q < g1; q += kYzThreads) {
    const int e = k.box[q] - pbase;
    const int i2 = e / n, i3 = e - i2 * n;
    const cplx<T> v = P[((i2 % N1) * N2 + i2 / N1) * LS + (i3 % N1) * N2 + i3 / N1];
    const cplx<T> xv = x[q];
    const T kr = kin[q];
    yv[q] = mk<T>(v.x * scale + kr * xv.x, v.y * scale + kr * xv.y);
  }
}

template <typename T>
static size_t yz_reg_lds(int n) {
  return sizeof(cplx<T>) * ((size_t)n * (n + 1) + n);
}

// (n, N1, N2) of the register plane transforms; false when not applicable
template <typename T>
static bool yz_reg_ok(const GridGeom& g) {
  if (g.n2 != g.n3) return false;
  if (yz_reg_lds<T>(g.n2) > kLdsMax) return false;
  switch (g.n2) {
#define X(nn, a, b) case nn:
    EAHP_YZREG_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

template <typename T>
void launch_inv_yz(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& pz,
                   const FftPlan& py, const cplx<T>* twz, const cplx<T>* twy, const cplx<T>* X, cplx<T>* Tb) {
  if (ncols <= 0) return;
  if (yz_reg_ok<T>(g)) {
    const size_t l = yz_reg_lds<T>(g.n2);
    dim3 grid(g.ns, ncols);
    switch (g.n2) {
#define X(nn, a, b)                                                                                             \
  case nn:                                                                                                      \
    HIPCK(hipFuncSetAttribute((const void*)k_inv_yz_reg<T, a, b>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              (int)l));                                                                         \
    hipLaunchKernelGGL((k_inv_yz_reg<T, a, b>), grid, dim3(kYzThreads), l, st, cm, g, twz, X, Tb);                \
    break;
      EAHP_YZREG_SIZES(X)
#undef X
      default:
        break;
    }
    HIPCK(hipGetLastError());
    return;
  }
  const size_t lds = plane_lds<T>(g);
  if (lds > kLdsMax) {
    // split plane: scatter + z-transform per block of z-lines, then the y-lines
    const int BZ = line_block(g.n3, sizeof(cplx<T>), 64 * 1024);
    const size_t lz = sizeof(cplx<T>) * ((size_t)BZ * g.n3 + g.n3);
    dim3 gz((g.n2 + BZ - 1) / BZ, g.ns, ncols);
    switch (pick_maxpts((int64_t)BZ * g.n3, 256)) {
#define CASE(M)                                                                                   \
  case M:                                                                                         \
    set_lds<T, M>((const void*)k_inv_z_sphere<T, M>, lz);                                        \
    hipLaunchKernelGGL((k_inv_z_sphere<T, M>), gz, dim3(256), lz, st, cm, g, BZ, pz, twz, X, Tb); \
    break;
      CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    }
    HIPCK(hipGetLastError());
    launch_lines<T>(st, Tb, g.ps, ncols * g.ns, g.n2, g.n3, 1, g.n3, py, twy, (T)1);
    return;
  }
  const int np = g.n2 * g.n3;
  const int nt = np >= 2048 ? 1024 : (np >= 512 ? 256 : 64);
  dim3 grid(g.ns, ncols);
  switch (pick_maxpts(np, nt)) {
#define CASE(M)                                                                                   \
  case M:                                                                                         \
    set_lds<T, M>((const void*)k_inv_yz<T, M>, lds);                                              \
    hipLaunchKernelGGL((k_inv_yz<T, M>), grid, dim3(nt), lds, st, cm, g, pz, py, twz, twy, X, Tb); \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
}

template <typename T>
void launch_fwd_yz(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& pz,
                   const FftPlan& py, const cplx<T>* twz, const cplx<T>* twy, const cplx<T>* Tb, const cplx<T>* X,
                   cplx<T>* HX) {
  if (ncols <= 0) return;
  const T scale = (T)(1.0 / ((double)g.n1 * g.n2 * g.n3));
  if (yz_reg_ok<T>(g)) {
    const size_t l = yz_reg_lds<T>(g.n2);
    dim3 grid(g.ns, ncols);
    switch (g.n2) {
#define X(nn, a, b)                                                                                             \
  case nn:                                                                                                      \
    HIPCK(hipFuncSetAttribute((const void*)k_fwd_yz_reg<T, a, b>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              (int)l));                                                                         \
    hipLaunchKernelGGL((k_fwd_yz_reg<T, a, b>), grid, dim3(kYzThreads), l, st, cm, g, twz, Tb, X, HX, scale);     \
    break;
      EAHP_YZREG_SIZES(X)
#undef X
      default:
        break;
    }
    HIPCK(hipGetLastError());
    return;
  }
  const size_t lds = plane_lds<T>(g);
  if (lds > kLdsMax) {
    // split plane: the y-lines in place on the slab, then z-transform + gather per block of z-lines
    launch_lines<T>(st, const_cast<cplx<T>*>(Tb), g.ps, ncols * g.ns, g.n2, g.n3, 1, g.n3, py, twy, (T)-1);
    const int BZ = line_block(g.n3, sizeof(cplx<T>), 64 * 1024);
    const size_t lz = sizeof(cplx<T>) * ((size_t)BZ * g.n3 + g.n3);
    dim3 gz((g.n2 + BZ - 1) / BZ, g.ns, ncols);
    switch (pick_maxpts((int64_t)BZ * g.n3, 256)) {
#define CASE(M)                                                                                                \
  case M:                                                                                                      \
    set_lds<T, M>((const void*)k_fwd_z_sphere<T, M>, lz);                                                     \
    hipLaunchKernelGGL((k_fwd_z_sphere<T, M>), gz, dim3(256), lz, st, cm, g, BZ, pz, twz, Tb, X, HX, scale); \
    break;
      CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    }
    HIPCK(hipGetLastError());
    return;
  }
  const int np = g.n2 * g.n3;
  const int nt = np >= 2048 ? 1024 : (np >= 512 ? 256 : 64);
  dim3 grid(g.ns, ncols);
  switch (pick_maxpts(np, nt)) {
#define CASE(M)                                                                                             \
  case M:                                                                                                   \
    set_lds<T, M>((const void*)k_fwd_yz<T, M>, lds);                                                        \
    hipLaunchKernelGGL((k_fwd_yz<T, M>), grid, dim3(nt), lds, st, cm, g, pz, py, twz, twy, Tb, X, HX, scale); \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
}

// The register x-kernels address a column's active planes through byte
// offsets: held in registers for the whole work-group where the extra
// registers cost no occupancy (offsets[a][j1]), else read per column from an
// LDS table of plane offsets (XOffsets<false>).
template <typename T, int N1, int N2, bool kDensity>
constexpr bool x_hoist_offsets() {
  constexpr int n = N1 * N2;
  if (kDensity) return !(n == 30 || n == 45 || n == 100 || n == 120 || n == 128 || n == 144);
  if (sizeof(T) == 4) return !(n == 54 || n == 60 || n == 75 || n == 80 || n == 81 || n == 100 || n == 120 || n == 128);
  return !(n == 27 || n == 30 || n == 32 || n == 45 || n == 100);
}
template <int JA, int N1, int N2, int G, bool kHoist>
struct XOffsets {
  uint32_t off[JA][N1];
  __device__ __forceinline__ void init(const uint32_t* soff, int grp, uint32_t posb) {
#pragma unroll
    for (int a = 0; a < JA; ++a) {
      const int j2 = grp + G * a;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) off[a][j1] = j2 < N2 ? soff[N2 * j1 + j2] + posb : kBufOob;
    }
  }
  __device__ __forceinline__ uint32_t get(const uint32_t*, int, uint32_t, int a, int j1) const { return off[a][j1]; }
};
template <int JA, int N1, int N2, int G>
struct XOffsets<JA, N1, N2, G, false> {
  __device__ __forceinline__ void init(const uint32_t*, int, uint32_t) {}
  __device__ __forceinline__ uint32_t get(const uint32_t* soff, int grp, uint32_t posb, int a, int j1) const {
    const int j2 = grp + G * a;
    return j2 < N2 ? soff[N2 * j1 + j2] + posb : kBufOob;
  }
};
// soff[i1] = byte offset of plane i1 in a column's slab, kBufOob if inactive;
// posb = the lane's byte offset within a plane, kBufOob past the last line.
// The host keeps the slab below kBufOob bytes, so soff + posb does not wrap
// and is out of range whenever either term is.
template <typename T>
__device__ __forceinline__ void x_plane_offsets(uint32_t* soff, int n1, const GridGeom& g, int lane) {
  for (int i = lane; i < n1; i += 64) soff[i] = kBufOob;
  __syncthreads();
  for (int s = lane; s < g.ns; s += 64) soff[g.plane_i1[s]] = (uint32_t)((int64_t)s * g.ps * (int64_t)sizeof(cplx<T>));
  __syncthreads();
}

// ------------------------------------------------------------------ x_local, register x-transform
// The same operation as k_x_local for n1 = N1 N2 (both products of at most two
// of 2, 3, 4, 5), with the x-transform as a four-step DFT in registers:
// j = N2 j1 + j2, k = k1 + N1 k2,
//   z(k1; j2) = w_n^{j2 k1} sum_j1 w_N1^{j1 k1} x(N2 j1 + j2),
//   y(k1 + N1 k2) = sum_j2 w_N2^{j2 k2} z(k1; j2).
// One wave per work-group, 16 (i2, i3) lines per wave, lane = line + 16 grp.
// Step A (the lane's j2 = grp + 4a): loads of the active planes straight from
// the slab (16 consecutive positions per plane; buffer loads, the inactive
// planes reading zero through the buffer's range check), size-N1 DFTs,
// twiddles, to
// LDS.  Step B (k1 = grp + 4b): size-N2 DFTs, times V_eff (held in registers
// for the work-group's columns), inverse size-N2 DFTs, twiddles, to LDS.
// Step A': inverse size-N1 DFTs, stores of the active planes.  An LDS location
// (k1, j2, line) is touched by one lane in steps A and A' and by one lane in
// step B, so the two barriers between the steps are the only ones.
template <typename T, int N1, int N2>
__global__ void __launch_bounds__(64) k_x_local_reg(int ncols, int cb, GridGeom g, const cplx<T>* __restrict__ twx,
                                                    const T* __restrict__ V, cplx<T>* __restrict__ Tb) {
  constexpr int n1 = N1 * N2, L = 16, G = 4;
  constexpr int JA = (N2 + G - 1) / G, KB = (N1 + G - 1) / G;
  __shared__ cplx<T> buf[n1 * L];
  __shared__ cplx<T> tw[n1];
  __shared__ uint32_t soff[n1];
  const int lane = threadIdx.x, t = lane & (L - 1), grp = lane >> 4;
  const int np = g.n2 * g.n3;
  const int pos = blockIdx.x * L + t;
  const bool valid = pos < np;
  const uint32_t posb = valid ? (uint32_t)pos * (uint32_t)sizeof(cplx<T>) : kBufOob;
  for (int i = lane; i < n1; i += 64) tw[i] = twx[i];
  x_plane_offsets<T>(soff, n1, g, lane);
  XOffsets<JA, N1, N2, G, x_hoist_offsets<T, N1, N2, false>()> xo;
  xo.init(soff, grp, posb);
  T vr[KB][N2];
#pragma unroll
  for (int b = 0; b < KB; ++b) {
    const int k1 = grp + G * b;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2)
      vr[b][k2] = (k1 < N1 && valid) ? V[(int64_t)(k1 + N1 * k2) * np + pos] : (T)0;
  }
  const uint32_t slab_bytes = (uint32_t)((int64_t)g.ns * g.ps * (int64_t)sizeof(cplx<T>));
  const int c0 = blockIdx.y * cb, c1 = min(ncols, c0 + cb);
  for (int c = c0; c < c1; ++c) {
    const __amdgpu_buffer_rsrc_t col = make_buf<T>(Tb + (int64_t)c * g.ns * g.ps, slab_bytes);
    cplx<T> u[JA][N1];
#pragma unroll
    for (int a = 0; a < JA; ++a)
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) u[a][j1] = buf_load<T>(col, xo.get(soff, grp, posb, a, j1));
#pragma unroll
    for (int a = 0; a < JA; ++a) {
      const int j2 = grp + G * a;
      if (j2 < N2) {
        RegFft<T, N1>::run(u[a], (T)1);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
          cplx<T> w = tw[j2 * k1];
          w.y = -w.y;  // exp(+2 pi i j2 k1 / n1)
          buf[(k1 * N2 + j2) * L + t] = k1 == 0 ? u[a][0] : cmul<T>(u[a][k1], w);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int k1 = grp + G * b;
      if (k1 < N1) {
        cplx<T> y[N2];
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) y[j2] = buf[(k1 * N2 + j2) * L + t];
        RegFft<T, N2>::run(y, (T)1);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) y[k2] = cscale<T>(y[k2], vr[b][k2]);
        RegFft<T, N2>::run(y, (T)-1);
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) buf[(k1 * N2 + j2) * L + t] = j2 == 0 ? y[0] : cmul<T>(y[j2], tw[j2 * k1]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < JA; ++a) {
      const int j2 = grp + G * a;
      if (j2 < N2) {
        cplx<T> x[N1];
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) x[k1] = buf[(k1 * N2 + j2) * L + t];
        RegFft<T, N1>::run(x, (T)-1);
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) buf_store(col, xo.get(soff, grp, posb, a, j1), x[j1]);
      }
    }
  }
}

// work-groups of k_x_local_reg<T, N1, N2> resident on the device at once
template <typename T, int N1, int N2>
static int x_local_concurrency() {
  static const int c = [] {
    int per = 0, dev = 0, ncu = 0;
    HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_x_local_reg<T, N1, N2>, 64, 0));
    HIPCK(hipGetDevice(&dev));
    HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    return std::max(1, per * ncu);
  }();
  return c;
}

// Columns per work-group.  The work-groups all take about the same time, so
// they run in rounds of `conc` (the resident ones); among up to 32 column
// chunks the count whose last round is fullest is taken (the first of equal
// ones: fewer chunks load V_eff fewer times).  At 90^3 (507 tiles of 16
// lines) and 128 columns that is 6 chunks of 22 columns, one round of 3042
// work-groups on 3072 slots.
static int x_local_columns(int ntiles, int ncols, int conc) {
  int best = 1;
  double beff = -1.0;
  for (int nch = 1; nch <= std::min(ncols, 32); ++nch) {
    const int64_t items = (int64_t)ntiles * nch;
    const int64_t rounds = (items + conc - 1) / conc;
    const double eff = (double)items / (double)(rounds * conc);
    if (eff > beff + 1e-3) {
      beff = eff;
      best = nch;
    }
  }
  return (ncols + best - 1) / best;
}

template <typename T>
static bool launch_x_local_reg(hipStream_t st, int ncols, const GridGeom& g, const cplx<T>* twx, const T* V,
                               cplx<T>* Tb) {
  const int np = g.n2 * g.n3;
  if ((int64_t)g.ns * g.ps * (int64_t)sizeof(cplx<T>) >= (int64_t)kBufOob) return false;
  const int ntiles = (np + 15) / 16;
  switch (g.n1) {
#define X(n, a, b)                                                                                           \
  case n: {                                                                                                  \
    const int cb = x_local_columns(ntiles, ncols, x_local_concurrency<T, a, b>());                           \
    const dim3 grid(ntiles, (ncols + cb - 1) / cb);                                                          \
    hipLaunchKernelGGL((k_x_local_reg<T, a, b>), grid, dim3(64), 0, st, ncols, cb, g, twx, V, Tb);             \
    HIPCK(hipGetLastError());                                                                                \
    return true;                                                                                             \
  }
    EAHP_XREG_SIZES(X)
#undef X
    default:
      return false;
  }
}

static int x_tile(int n1, int np, size_t per_elem, size_t budget) {
  int tile = 64;
  while (tile > 8 && (size_t)n1 * tile * per_elem > budget) tile /= 2;
  if (tile > np) tile = np;
  return tile;
}

template <typename T>
void launch_x_local(hipStream_t st, int ncols, const GridGeom& g, const FftPlan& px, const cplx<T>* twx,
                    const T* V, cplx<T>* Tb) {
  if (ncols <= 0) return;
  if (launch_x_local_reg<T>(st, ncols, g, twx, V, Tb)) return;
  const int np = g.n2 * g.n3;
  // LDS per work-group bounds how many work-groups share a CU, and with them
  // how much of the slab traffic is in flight: about 36 KB gives four
  const int tile = x_tile(g.n1, np, sizeof(cplx<T>) + sizeof(T), 36 * 1024);
  const size_t lds = (size_t)g.n1 * tile * (sizeof(cplx<T>) + sizeof(T)) + g.n1 * sizeof(cplx<T>);
  const int nt = g.n1 * tile >= 2048 ? 512 : 256;
  const int ntiles = (np + tile - 1) / tile;
  // columns per work-group: enough work-groups to fill the chip, V reused by the chunk
  int cb = 16;
  while (cb > 1 && (int64_t)ntiles * ((ncols + cb - 1) / cb) < 1024) cb /= 2;
  dim3 grid(ntiles, (ncols + cb - 1) / cb);
  switch (pick_maxpts((int64_t)g.n1 * tile, nt)) {
#define CASE(M)                                                                                       \
  case M:                                                                                             \
    set_lds<T, M>((const void*)k_x_local<T, M>, lds);                                                 \
    hipLaunchKernelGGL((k_x_local<T, M>), grid, dim3(nt), lds, st, ncols, cb, g, tile, px, twx, V, Tb); \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
}

// rho[i] (+)= sum over the column groups of part[grp][i], groups in order
__global__ void __launch_bounds__(256) k_sum_groups(int64_t n, int ngrp, const double* __restrict__ part,
                                                    int64_t sgrp, double* __restrict__ rho, int accumulate) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int gi = 0; gi < ngrp; ++gi) acc += part[gi * sgrp + i];
    rho[i] = accumulate ? rho[i] + acc : acc;
  }
}

// x_density with the register x-transform of k_x_local_reg (steps A and B of
// the inverse transform), w_k f |psi|^2 / Omega accumulated in registers over
// the work-group's columns, in column order.
template <int N1, int N2>
__global__ void __launch_bounds__(64) k_x_density_reg(ColMap cm, int ncols, int cpg, GridGeom g,
                                                      const z64* __restrict__ twx, const z64* __restrict__ Tb,
                                                      double occ_over_omega, double* __restrict__ rho, int accumulate,
                                                      int64_t sgrp) {
  constexpr int n1 = N1 * N2, L = 16, G = 4;
  constexpr int JA = (N2 + G - 1) / G, KB = (N1 + G - 1) / G;
  __shared__ z64 buf[n1 * L];
  __shared__ z64 tw[n1];
  __shared__ uint32_t soff[n1];
  const int lane = threadIdx.x, t = lane & (L - 1), grp = lane >> 4;
  const int np = g.n2 * g.n3;
  const int pos = blockIdx.x * L + t;
  const bool valid = pos < np;
  const uint32_t posb = valid ? (uint32_t)pos * (uint32_t)sizeof(z64) : kBufOob;
  for (int i = lane; i < n1; i += 64) tw[i] = twx[i];
  x_plane_offsets<double>(soff, n1, g, lane);
  XOffsets<JA, N1, N2, G, x_hoist_offsets<double, N1, N2, true>()> xo;
  xo.init(soff, grp, posb);
  double acc[KB][N2];
#pragma unroll
  for (int b = 0; b < KB; ++b)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) acc[b][k2] = 0.0;
  const uint32_t slab_bytes = (uint32_t)((int64_t)g.ns * g.ps * (int64_t)sizeof(z64));
  const int cbeg = blockIdx.y * cpg, cend = min(ncols, cbeg + cpg);
  rho += blockIdx.y * sgrp;
  for (int c = cbeg; c < cend; ++c) {
    int64_t base;
    const KDesc& k = col_kd(cm, c, base);
    const double wgt = k.w * occ_over_omega;
    const __amdgpu_buffer_rsrc_t col = make_buf<double>(Tb + (int64_t)c * g.ns * g.ps, slab_bytes);
    z64 u[JA][N1];
#pragma unroll
    for (int a = 0; a < JA; ++a)
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) u[a][j1] = buf_load<double>(col, xo.get(soff, grp, posb, a, j1));
#pragma unroll
    for (int a = 0; a < JA; ++a) {
      const int j2 = grp + G * a;
      if (j2 < N2) {
        RegFft<double, N1>::run(u[a], 1.0);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
          z64 w = tw[j2 * k1];
          w.y = -w.y;
          buf[(k1 * N2 + j2) * L + t] = k1 == 0 ? u[a][0] : cmul<double>(u[a][k1], w);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int k1 = grp + G * b;
      if (k1 < N1) {
        z64 y[N2];
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) y[j2] = buf[(k1 * N2 + j2) * L + t];
        RegFft<double, N2>::run(y, 1.0);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) acc[b][k2] += wgt * (y[k2].x * y[k2].x + y[k2].y * y[k2].y);
      }
    }
    __syncthreads();  // the next column's step A writes locations read here by other lanes
  }
  if (valid) {
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int k1 = grp + G * b;
      if (k1 < N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          double* d = rho + (int64_t)(k1 + N1 * k2) * np + pos;
          *d = accumulate ? *d + acc[b][k2] : acc[b][k2];
        }
      }
    }
  }
}

static bool launch_x_density_reg(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const z64* twx,
                                 const z64* Tb, double occ_over_omega, double* rho, int accumulate, DevMem& part) {
  if ((int64_t)g.ns * g.ps * (int64_t)sizeof(z64) >= (int64_t)kBufOob) return false;
  switch (g.n1) {
#define X(n, a, b) case n:
    EAHP_XREG_SIZES(X)
#undef X
    break;
    default:
      return false;
  }
  const int np = g.n2 * g.n3;
  const int ntiles = (np + 15) / 16;
  // column groups until there are >= 2048 single-wave work-groups, while the
  // partial densities (written and read once more) stay under a fifth of the
  // slab bytes; each group sums into its own partial, reduced in a fixed order
  int ngrp = 1;
  while (ngrp < 16 && (int64_t)ntiles * ngrp < 2048 && (int64_t)(2 * ngrp) * g.n1 * 5 <= (int64_t)ncols * g.ns)
    ngrp *= 2;
  const int cpg = (ncols + ngrp - 1) / ngrp;
  ngrp = (ncols + cpg - 1) / cpg;
  const int64_t Ng = (int64_t)g.n1 * np;
  double* dst = rho;
  int acc_k = accumulate;
  if (ngrp > 1) {
    part.ensure(sizeof(double) * Ng * ngrp);
    dst = part.as<double>();
    acc_k = 0;
  }
  dim3 grid(ntiles, ngrp);
  switch (g.n1) {
#define X(n, a, b)                                                                                                 \
  case n:                                                                                                          \
    hipLaunchKernelGGL((k_x_density_reg<a, b>), grid, dim3(64), 0, st, cm, ncols, cpg, g, twx, Tb, occ_over_omega, \
                       dst, acc_k, Ng);                                                                            \
    break;
    EAHP_XREG_SIZES(X)
#undef X
    default:
      break;
  }
  HIPCK(hipGetLastError());
  if (ngrp > 1) {
    hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)std::min<int64_t>(2048, (Ng + 255) / 256)), dim3(256), 0, st, Ng,
                       ngrp, part.as<double>(), Ng, rho, accumulate);
    HIPCK(hipGetLastError());
  }
  return true;
}

void launch_x_density(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& px,
                      const z64* twx, const z64* Tb, double occ_over_omega, double* rho, int accumulate,
                      DevMem& part) {
  if (launch_x_density_reg(st, cm, ncols, g, twx, Tb, occ_over_omega, rho, accumulate, part)) return;
  const int np = g.n2 * g.n3;
  const int tile = std::min(32, x_tile(g.n1, np, sizeof(z64), 48 * 1024));
  const size_t lds = (size_t)g.n1 * tile * sizeof(z64) + g.n1 * sizeof(z64);
  const int nt = 256;
  const int ntiles = (np + tile - 1) / tile;
  // column groups until the grid fills the chip, while the partial densities
  // (written and read once more) stay under a tenth of the slab bytes; each
  // group sums into its own partial, reduced afterwards in a fixed order
  int ngrp = 1;
  while (ngrp < 16 && (int64_t)ntiles * ngrp < 1024 && (int64_t)(2 * ngrp) * g.n1 * 10 <= (int64_t)ncols * g.ns)
    ngrp *= 2;
  const int cpg = (ncols + ngrp - 1) / ngrp;
  ngrp = (ncols + cpg - 1) / cpg;
  const int64_t Ng = (int64_t)g.n1 * np;
  double* dst = rho;
  int acc_k = accumulate;
  if (ngrp > 1) {
    part.ensure(sizeof(double) * Ng * ngrp);
    dst = part.as<double>();
    acc_k = 0;
  }
  switch (pick_maxpts((int64_t)g.n1 * tile, nt)) {
#define CASE(M)                                                                                                 \
  case M:                                                                                                       \
    set_lds<double, M>((const void*)k_x_density<M>, lds);                                                      \
    hipLaunchKernelGGL((k_x_density<M>), dim3(ntiles, ngrp), dim3(nt), lds, st, cm, ncols, cpg, g, tile, px, twx, \
                       Tb, occ_over_omega, dst, acc_k, Ng);                                                     \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
  if (ngrp > 1) {
    hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)std::min<int64_t>(2048, (Ng + 255) / 256)), dim3(256), 0, st, Ng,
                       ngrp, part.as<double>(), Ng, rho, accumulate);
    HIPCK(hipGetLastError());
  }
}

template void launch_inv_yz<double>(hipStream_t, const ColMap&, int, const GridGeom&, const FftPlan&, const FftPlan&,
                                    const z64*, const z64*, const z64*, z64*);
template void launch_inv_yz<float>(hipStream_t, const ColMap&, int, const GridGeom&, const FftPlan&, const FftPlan&,
                                   const c32*, const c32*, const c32*, c32*);
template void launch_fwd_yz<double>(hipStream_t, const ColMap&, int, const GridGeom&, const FftPlan&, const FftPlan&,
                                    const z64*, const z64*, const z64*, const z64*, z64*);
template void launch_fwd_yz<float>(hipStream_t, const ColMap&, int, const GridGeom&, const FftPlan&, const FftPlan&,
                                   const c32*, const c32*, const c32*, const c32*, c32*);
template void launch_x_local<double>(hipStream_t, int, const GridGeom&, const FftPlan&, const z64*, const double*,
                                     z64*);
template void launch_x_local<float>(hipStream_t, int, const GridGeom&, const FftPlan&, const c32*, const float*,
                                    c32*);

// ------------------------------------------------------------------ full-box FFT (potentials)
template <int MAXPTS>
__global__ void __launch_bounds__(1024) k_box_yz(int n2, int n3, FftPlan pz, FftPlan py, const z64* twz,
                                                 const z64* twy, z64* box, double sg) {
  extern __shared__ unsigned char smem_raw[];
  const int np = n2 * n3;
  z64* pl = reinterpret_cast<z64*>(smem_raw);
  z64* tz = pl + np;
  z64* ty = tz + n3;
  z64* p0 = box + (int64_t)blockIdx.x * np;
  for (int i = threadIdx.x; i < np; i += blockDim.x) pl[i] = p0[i];
  for (int i = threadIdx.x; i < n3; i += blockDim.x) tz[i] = twz[i];
  for (int i = threadIdx.x; i < n2; i += blockDim.x) ty[i] = twy[i];
  __syncthreads();
  lds_fft<double, MAXPTS>(pl, Lines{n3, 1, n2, n3, 0}, pz, tz, sg);
  lds_fft<double, MAXPTS>(pl, Lines{n2, n3, n3, 1, 1}, py, ty, sg);
  for (int i = threadIdx.x; i < np; i += blockDim.x) p0[i] = pl[i];
}

template <int MAXPTS>
__global__ void __launch_bounds__(512) k_box_x(int n1, int np, int tile, FftPlan px, const z64* twx, z64* box,
                                               double sg) {
  extern __shared__ unsigned char smem_raw[];
  z64* buf = reinterpret_cast<z64*>(smem_raw);
  z64* tw = buf + n1 * tile;
  const int t0 = blockIdx.x * tile;
  const int cnt = min(tile, np - t0);
  for (int i = threadIdx.x; i < n1; i += blockDim.x) tw[i] = twx[i];
  for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) {
    const int i1 = e / tile, t = e - i1 * tile;
    buf[e] = t < cnt ? box[(int64_t)i1 * np + t0 + t] : mk<double>(0, 0);
  }
  __syncthreads();
  lds_fft<double, MAXPTS>(buf, Lines{n1, tile, tile, 1, 1}, px, tw, sg);
  for (int e = threadIdx.x; e < n1 * tile; e += blockDim.x) {
    const int i1 = e / tile, t = e - i1 * tile;
    if (t < cnt) box[(int64_t)i1 * np + t0 + t] = buf[e];
  }
}

void launch_box_fft(hipStream_t st, int n1, int n2, int n3, const FftPlan p[3], const z64* const tw[3], z64* box,
                    double sign) {
  const int np = n2 * n3;
  const size_t lds = sizeof(z64) * ((size_t)np + n2 + n3);
  const int nt = np >= 2048 ? 1024 : (np >= 512 ? 256 : 64);
  if (lds > kLdsMax) {
    // split plane: z-lines, then y-lines, of every x-plane
    launch_lines<double>(st, box, np, n1, n3, 1, n3, n2, p[2], tw[2], sign);
    launch_lines<double>(st, box, np, n1, n2, n3, 1, n3, p[1], tw[1], sign);
  } else
  switch (pick_maxpts(np, nt)) {
#define CASE(M)                                                                                                  \
  case M:                                                                                                        \
    set_lds<double, M>((const void*)k_box_yz<M>, lds);                                                           \
    hipLaunchKernelGGL((k_box_yz<M>), dim3(n1), dim3(nt), lds, st, n2, n3, p[2], p[1], tw[2], tw[1], box, sign); \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
  const int tile = x_tile(n1, np, sizeof(z64), 64 * 1024);
  const size_t lds2 = (size_t)n1 * tile * sizeof(z64) + n1 * sizeof(z64);
  const int nt2 = 256;
  switch (pick_maxpts((int64_t)n1 * tile, nt2)) {
#define CASE(M)                                                                                                   \
  case M:                                                                                                         \
    set_lds<double, M>((const void*)k_box_x<M>, lds2);                                                            \
    hipLaunchKernelGGL((k_box_x<M>), dim3((np + tile - 1) / tile), dim3(nt2), lds2, st, n1, np, tile, p[0], tw[0], \
                       box, sign);                                                                                \
    break;
    CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
  HIPCK(hipGetLastError());
}

// ------------------------------------------------------------------ potentials
__global__ void k_rho_to_box(int64_t Ng, const double* rho, z64* box) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ng; i += (int64_t)gridDim.x * blockDim.x)
    box[i] = mk<double>(rho[i], 0.0);
}
void launch_rho_to_box(hipStream_t st, int64_t Ng, const double* rho, z64* box) {
  hipLaunchKernelGGL(k_rho_to_box, dim3(2048), dim3(256), 0, st, Ng, rho, box);
  HIPCK(hipGetLastError());
}

struct Mat3 {
  double b[9];
};

__device__ __forceinline__ int freq_of(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// box holds the forward DFT of rho (no 1/N_g); becomes V_H(G) = 4 pi rho^(G)/|G|^2
__global__ void k_hartree_g(int n1, int n2, int n3, Mat3 B, z64* box) {
  const int64_t Ng = (int64_t)n1 * n2 * n3;
  const double sc = 4.0 * M_PI / (double)Ng;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ng; i += (int64_t)gridDim.x * blockDim.x) {
    const int i3 = (int)(i % n3);
    const int i2 = (int)((i / n3) % n2);
    const int i1 = (int)(i / ((int64_t)n2 * n3));
    const double m1 = freq_of(i1, n1), m2 = freq_of(i2, n2), m3 = freq_of(i3, n3);
    const double gx = B.b[0] * m1 + B.b[3] * m2 + B.b[6] * m3;
    const double gy = B.b[1] * m1 + B.b[4] * m2 + B.b[7] * m3;
    const double gz = B.b[2] * m1 + B.b[5] * m2 + B.b[8] * m3;
    const double g2 = gx * gx + gy * gy + gz * gz;
    const z64 v = box[i];
    const double f = (i == 0) ? 0.0 : sc / g2;
    box[i] = mk<double>(v.x * f, v.y * f);
  }
}
void launch_hartree_g(hipStream_t st, int n1, int n2, int n3, const double* B, z64* box) {
  Mat3 m;
  for (int i = 0; i < 9; ++i) m.b[i] = B[i];
  hipLaunchKernelGGL(k_hartree_g, dim3(2048), dim3(256), 0, st, n1, n2, n3, m, box);
  HIPCK(hipGetLastError());
}

// Veff = Vion + VH + Vx;  partial[b*3 + {0,1,2}] = block sums of Vion rho, VH rho / 2, e_x
__global__ void __launch_bounds__(256) k_veff(int64_t Ng, const double* rho, const double* vion, const z64* vh,
                                              int terms, double cx, double* veff, float* veff32, double* partial) {
  __shared__ double sh[16];
  double s0 = 0, s1 = 0, s2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ng; i += (int64_t)gridDim.x * blockDim.x) {
    const double r = fmax(rho[i], 0.0);
    const double vi = (terms & EAHP_TERM_ION) ? vion[i] : 0.0;
    const double h = (terms & EAHP_TERM_HARTREE) ? vh[i].x : 0.0;
    double vx = 0.0, ex = 0.0;
    if (terms & EAHP_TERM_XC) {
      vx = -cx * cbrt(r);
      ex = 0.75 * r * vx;
    }
    const double v = vi + h + vx;
    veff[i] = v;
    if (veff32) veff32[i] = (float)v;
    s0 += vi * rho[i];
    s1 += 0.5 * h * rho[i];
    s2 += ex;
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x * 3 + 0] = s0;
    partial[blockIdx.x * 3 + 1] = s1;
    partial[blockIdx.x * 3 + 2] = s2;
  }
}
void launch_veff(hipStream_t st, int64_t Ng, const double* rho, const double* vion, const z64* vh_box, int terms,
                 double* veff, float* veff32, double* partial3, int nblocks) {
  const double cx = std::cbrt(3.0 / M_PI);  // Slater: V_x = -(3 rho / pi)^(1/3)
  hipLaunchKernelGGL(k_veff, dim3(nblocks), dim3(256), 0, st, Ng, rho, vion, vh_box, terms, cx, veff, veff32,
                     partial3);
  HIPCK(hipGetLastError());
}

__global__ void k_real_part(int64_t Ng, const z64* box, double scale, double* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ng; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = box[i].x * scale;
}
void launch_real_part(hipStream_t st, int64_t Ng, const z64* box, double scale, double* out) {
  hipLaunchKernelGGL(k_real_part, dim3(2048), dim3(256), 0, st, Ng, box, scale, out);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
