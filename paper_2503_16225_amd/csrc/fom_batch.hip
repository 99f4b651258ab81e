// Algorithm 4 (the preconditioned block FOM of the metric solve, Appendix A)
// on all k-points of a problem at once.  The problem lives on the product
// manifold (Sec. 5.1): H is block diagonal over k and every k-point has its
// own Sylvester equation H_k X_k - X_k Sigma_k = Phi_k, its own Krylov space
// and its own stopping test.  Here the k-blocks are padded to a common leading
// dimension ld (rows n_k.. hold zeros), so that every product of the method is
// one batched launch over the k-points, the H-applies of each stage are one
// launch over the columns of all k-points still iterating, and the host
// synchronises once per stage for all k-points (norms and ranks).
//
// A direction that deflates in the rank-revealing step (pivot below the
// cut-off) enters the basis as a zero column whose projected diagonal entry is
// set to a constant above the spectrum: the column is decoupled from the rest,
// its coefficient in the projected solution is zero, and the Galerkin solution
// on the retained directions is that of the one-k-point method.  A k-point
// that has stopped contributes zero blocks from then on, and its solution is
// formed when it stops.  The projected problems A_j Y - Y Sigma = C_j are
// solved in the eigenbasis of Sigma, through batched Householder tridiagonal
// reductions of A_j and shifted tridiagonal solves (all k-points in the same
// launches) up to q = 512 and through eigendecompositions of A_j beyond.
#include <algorithm>
#include <cmath>
#include <vector>

#include "devcommon.h"
#include "ops.h"
#include "setup.h"

namespace eahp {

namespace {

// largest projected order of the batched tridiagonal solve (larger ones go
// through eigendecompositions, one k-point at a time)
constexpr int kTriMax = 512;

template <typename T>
__global__ void k_frame_to_pad(int p, const KDesc* __restrict__ kd, const z64* __restrict__ src, double scale,
                               cplx<T>* __restrict__ dst, int64_t ld) {
  const int k = blockIdx.y;
  const KDesc K = kd[k];
  const int64_t tot = ld * p;
  const z64* s = src + (int64_t)p * K.off;
  cplx<T>* d = dst + (int64_t)k * tot;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ld, r = e - j * ld;
    cplx<T> v = mk<T>(0, 0);
    if (r < K.npw) {
      const z64 x = s[j * K.npw + r];
      v = mk<T>((T)(scale * x.x), (T)(scale * x.y));
    }
    d[e] = v;
  }
}

// dst_k[r, j] = src_k[r, j] / (kin_k[r] + alpha_k[j]) on the padded blocks
template <typename T>
__global__ void k_tpa_pad(int p, int64_t ld, const double* __restrict__ kinp, const double* __restrict__ alpha,
                          const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst) {
  const int k = blockIdx.y;
  const int64_t tot = ld * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ld, r = e - j * ld;
    const double f = 1.0 / (kinp[k * ld + r] + alpha[(int64_t)k * p + j]);
    const cplx<T> x = src[k * tot + e];
    dst[k * tot + e] = mk<T>((T)(f * x.x), (T)(f * x.y));
  }
}

// squared norms of all nk p padded columns (FP64 sums), one wave per column
template <typename T>
__global__ void __launch_bounds__(256) k_col_norms(int ncols, int64_t ld, const cplx<T>* __restrict__ X,
                                                   double* __restrict__ out) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= ncols) return;
  const cplx<T>* x = X + (int64_t)c * ld;
  double s = 0;
  for (int64_t r = lane; r < ld; r += 64) s += (double)x[r].x * x[r].x + (double)x[r].y * x[r].y;
  s = warp_sum(s);
  if (lane == 0) out[c] = s;
}

// zero the padded blocks of the k-points whose flag is 0
template <typename T>
__global__ void k_mask_blocks(int64_t per, const int* __restrict__ live, cplx<T>* X, int64_t stride) {
  const int k = blockIdx.y;
  if (live[k]) return;
  cplx<T>* x = X + (int64_t)k * stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = mk<T>(0, 0);
}

template <typename T>
__global__ void k_zero_cols(int64_t ld, int ncols, cplx<T>* X, int64_t stride) {
  const int k = blockIdx.y;
  const int64_t per = ld * ncols;
  cplx<T>* x = X + (int64_t)k * stride;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x)
    x[e] = mk<T>(0, 0);
}

// the deflated columns of the new block (beyond rank[k]) get a decoupled
// diagonal entry `big` in A_k
__global__ void k_fix_deflated(int q0, int ncols, const int* __restrict__ rank, z64* A, int64_t lda, int64_t sA,
                               double big) {
  const int k = blockIdx.x;
  for (int c = rank[k] + threadIdx.x; c < ncols; c += blockDim.x)
    A[k * sA + (int64_t)(q0 + c) * (lda + 1)] = mk<double>(big, 0.0);
}

// Mirror A_k[0:q, q:q+r] into A_k[q:q+r, 0:q] (conjugate transpose) for every k
__global__ void k_border_mirror_b(int q, int r, z64* A, int64_t lda, int64_t sA) {
  z64* a = A + blockIdx.y * sA;
  const int tot = q * r;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += gridDim.x * blockDim.x) {
    const int i = e % q, j = e / q;
    const z64 v = a[i + (int64_t)(q + j) * lda];
    a[(q + j) + (int64_t)i * lda] = mk<double>(v.x, -v.y);
  }
}

// Y_k[i, l] /= (w_k[i] - s_k[l])
__global__ void k_sylv_divide_b(int q, int p, const double* w, int64_t sw, const double* s, z64* Y, int64_t sY) {
  const int k = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q * p; e += gridDim.x * blockDim.x) {
    const int i = e % q, l = e / q;
    const double d = w[k * sw + i] - s[(int64_t)k * p + l];
    z64& y = Y[k * sY + e];
    y = mk<double>(y.x / d, y.y / d);
  }
}

// batched copies between precisions / leading dimensions (rows x cols per k)
template <typename S, typename D>
__global__ void k_conv_b(int rows, int cols, const S* src, int64_t lds, int64_t sS, D* dst, int64_t ldd, int64_t sD) {
  const int k = blockIdx.y;
  const int64_t tot = (int64_t)rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / rows, i = e - j * rows;
    const S v = src[k * sS + i + j * lds];
    dst[k * sD + i + j * ldd].x = v.x;
    dst[k * sD + i + j * ldd].y = v.y;
  }
}

template <typename S, typename D>
void conv_b(hipStream_t st, int rows, int cols, const S* src, int64_t lds, int64_t sS, D* dst, int64_t ldd, int64_t sD,
            int batch) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return;
  const int nb = (int)std::min<int64_t>(256, ((int64_t)rows * cols + 255) / 256);
  hipLaunchKernelGGL((k_conv_b<S, D>), dim3(nb, batch), dim3(256), 0, st, rows, cols, src, lds, sS, dst, ldd, sD);
  HIPCK(hipGetLastError());
}

unsigned nblk(int64_t n) { return (unsigned)std::min<int64_t>(1024, (n + 255) / 256); }

// X_k = scale Phi_k + (V Y)_k for the k-points k = list[blockIdx.y] (stacked
// frames; V Y padded, block k at k sF with leading dimension ld).  The product
// is rounded, then the sum (contraction into a fused multiply-add is off), as
// in the separate scaling and accumulation of a single k-point.
template <typename T>
__global__ void k_pad_to_frame_x(int p, const KDesc* __restrict__ kd, const int* __restrict__ list,
                                 const cplx<T>* __restrict__ XP, int64_t ld, int64_t sF, const z64* __restrict__ Phi,
                                 double scale, z64* __restrict__ X) {
#pragma clang fp contract(off)
  const int k = list[blockIdx.y];
  const int64_t n = kd[k].npw, o = (int64_t)p * kd[k].off, tot = n * p;
  const cplx<T>* xp = XP + (int64_t)k * sF;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / n, r = e - j * n;
    const cplx<T> v = xp[j * ld + r];
    const z64 f = Phi[o + e];
    const double tx = scale * f.x, ty = scale * f.y;
    X[o + e] = mk<double>(tx + (double)v.x, ty + (double)v.y);
  }
}

// Y_k[i, l] *= s_k[l]
__global__ void k_scale_cols_b(int q, int p, const double* s, z64* Y) {
  const int k = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q * p; e += gridDim.x * blockDim.x) {
    const int l = e / q;
    const double f = s[(int64_t)k * p + l];
    z64& y = Y[(int64_t)k * q * p + e];
    y = mk<double>(y.x * f, y.y * f);
  }
}

__global__ void k_fill_d(double* x, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

template <typename T>
struct Batch {
  using CT = cplx<T>;
  eahp_problem* pb;
  hipStream_t st;
  FomBatchWork& w;
  int p, nk;
  int64_t ld, pp, sF;
  int qcap() const { return w.qcap; }
  int64_t sV() const { return ld * w.qcap; }
  CT* V() const { return w.V.as<CT>(); }
  CT* W() const { return w.W.as<CT>(); }
  z64* A() const { return w.A.as<z64>(); }
  z64* Cj() const { return w.Cj.as<z64>(); }

  // C_k (a x b, ld ldc, stride sC, FP64) = A_k^H B_k over the ld padded rows
  void gram(int a, int b, const CT* Am, int64_t sA, const CT* Bm, int64_t sB, z64* C, int64_t ldc, int64_t sC) {
    if constexpr (sizeof(T) == 8) {
      gemm_hn<double>(st, ld, a, b, Am, ld, Bm, ld, C, ldc, 1.0, 0.0, pb->ws.gemm_part, nk, sA, sB, sC);
    } else {
      w.stage.ensure(sizeof(CT) * (size_t)a * b * nk);
      gemm_hn<float>(st, ld, a, b, Am, ld, Bm, ld, w.stage.as<CT>(), a, 1.0, 0.0, pb->ws.gemm_part, nk, sA, sB,
                     (int64_t)a * b);
      conv_b(st, a, b, w.stage.as<CT>(), a, (int64_t)a * b, C, ldc, sC, nk);
    }
  }

  // grow the Krylov blocks (V, W, A, Cj) to hold `need` columns, keeping q_used
  void grow(int need, int q_used) {
    if (need <= w.qcap) return;
    const int old = w.qcap;
    const int cap = std::max(need, 2 * old);
    DevMem V2, W2, A2, C2;
    V2.alloc(sizeof(CT) * (size_t)ld * cap * nk);
    W2.alloc(sizeof(CT) * (size_t)ld * cap * nk);
    A2.alloc(sizeof(z64) * (size_t)cap * cap * nk);
    C2.alloc(sizeof(z64) * (size_t)cap * p * nk);
    if (old > 0 && q_used > 0) {
      HIPCK(hipMemcpy2DAsync(V2.p, sizeof(CT) * ld * cap, w.V.p, sizeof(CT) * ld * old, sizeof(CT) * ld * q_used, nk,
                             hipMemcpyDeviceToDevice, st));
      HIPCK(hipMemcpy2DAsync(W2.p, sizeof(CT) * ld * cap, w.W.p, sizeof(CT) * ld * old, sizeof(CT) * ld * q_used, nk,
                             hipMemcpyDeviceToDevice, st));
      for (int k = 0; k < nk; ++k) {
        HIPCK(hipMemcpy2DAsync(A2.as<z64>() + (size_t)k * cap * cap, sizeof(z64) * cap,
                               w.A.as<z64>() + (size_t)k * old * old, sizeof(z64) * old, sizeof(z64) * q_used, q_used,
                               hipMemcpyDeviceToDevice, st));
        HIPCK(hipMemcpy2DAsync(C2.as<z64>() + (size_t)k * cap * p, sizeof(z64) * cap,
                               w.Cj.as<z64>() + (size_t)k * old * p, sizeof(z64) * old, sizeof(z64) * q_used, p,
                               hipMemcpyDeviceToDevice, st));
      }
      HIPCK(hipStreamSynchronize(st));  // the old buffers are freed below
    }
    std::swap(w.V, V2);
    std::swap(w.W, W2);
    std::swap(w.A, A2);
    std::swap(w.Cj, C2);
    w.qcap = cap;
  }

  // orthonormal basis of span(R_k) by pivoted CholQR twice, into dest (stride
  // sD, ld ld); columns beyond the rank are zero.  Returns the ranks (host);
  // rank (device) holds them too.
  std::vector<int> rrqr(const CT* R, CT* dest, int64_t sD, double tol) {
    z64* G = w.Gm64.as<z64>();
    z64* PU64 = w.PU64.as<z64>();
    int* piv = w.piv.as<int>();
    int* rank = w.rank.as<int>();
    CT* tmp = w.Tmp.as<CT>();
    auto pu = [&]() -> const CT* {
      if constexpr (sizeof(T) == 8) {
        return PU64;
      } else {
        conv_b(st, p, p, PU64, p, pp, w.PU.as<CT>(), p, pp, nk);
        return w.PU.as<CT>();
      }
    };
    gram(p, p, R, sF, R, sF, G, p, pp);
    pchol_inv_batched(st, p, G, p, pp, tol, piv, rank, PU64, p, pp, nk, w.chol);
    gemm_nn<T>(st, ld, p, p, R, ld, pu(), p, 0, tmp, ld, 1.0, 0.0, 0.0, nk, sF, pp, sF);
    gram(p, p, tmp, sF, tmp, sF, G, p, pp);
    pchol_inv_batched(st, p, G, p, pp, 0.0, piv, rank, PU64, p, pp, nk, w.chol);
    gemm_nn<T>(st, ld, p, p, tmp, ld, pu(), p, 0, dest, ld, 1.0, 0.0, 0.0, nk, sF, pp, sD);
    std::vector<int> r(nk);
    HIPCK(hipMemcpyAsync(r.data(), rank, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    return r;
  }

  // per-k squared norms of the padded blocks of X (host)
  std::vector<double> norms(const CT* Xp) {
    const int ncols = nk * p;
    hipLaunchKernelGGL(k_col_norms<T>, dim3((ncols + 3) / 4), dim3(256), 0, st, ncols, ld, Xp, w.norms.as<double>());
    HIPCK(hipGetLastError());
    std::vector<double> c(ncols), out(nk, 0.0);
    HIPCK(hipMemcpyAsync(c.data(), w.norms.p, sizeof(double) * ncols, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < p; ++j) out[k] += c[(size_t)k * p + j];
    return out;
  }

  // host -> device without waiting: every target has its own slot of the
  // pinned stage, rewritten only after a later synchronisation of the stream
  // (each FOM iteration synchronises on its residual norms and ranks)
  void upload(DevMem& d, const std::vector<int>& h, int slot) {
    int* s = w.hstage.as<int>() + (size_t)slot * nk;
    std::copy(h.begin(), h.end(), s);
    HIPCK(hipMemcpyAsync(d.p, s, sizeof(int) * h.size(), hipMemcpyHostToDevice, st));
  }

  // H V for the columns [q0, q0 + p) of the k-points in `act` (others: zero)
  void apply_H(int q0, const std::vector<int>& act) {
    hipLaunchKernelGGL(k_zero_cols<T>, dim3(nblk(ld * p), nk), dim3(256), 0, st, ld, p, W() + (int64_t)q0 * ld, sV());
    HIPCK(hipGetLastError());
    if (act.empty()) return;
    upload(w.kmap, act, 1);
    apply_H_padded<T>(pb, (int)act.size(), w.kmap.as<int>(), act.data(), p, V() + (int64_t)q0 * ld,
                      W() + (int64_t)q0 * ld, ld, sV());
  }
};

}  // namespace

template <typename T>
void fom_batch(eahp_problem* pb, const z64* Phi, const z64* R, const double* lw, const z64* lU, double mu, double rtol,
               int maxit, double rank_tol, z64* X, std::vector<FomInfo>& info) {
  using CT = cplx<T>;
  hipStream_t st = pb->ctx->stream;
  FomBatchWork& w = sizeof(T) == 8 ? pb->arena->fb64 : pb->arena->fb32;
  const int p = pb->p, nk = pb->nk;
  if (p > 128) fail(EAHP_EINVAL, "batched metric solve: p > 128");
  const int64_t ld = (pb->nmax + 15) / 16 * 16;
  Batch<T> b{pb, st, w, p, nk, ld, (int64_t)p * p, ld * p};
  const int64_t pp = b.pp, sF = b.sF;
  const double big = 2.0 * pb->ecut + 100.0;  // above every eigenvalue of the projected H
  info.assign(nk, FomInfo{});
  // the padded kinetic energies (pad 1: the padded rows of every operand are zero)
  if (w.ld != ld) {
    w.kinp.alloc(sizeof(double) * ld * nk);
    hipLaunchKernelGGL(k_fill_d, dim3(nblk(ld * nk)), dim3(256), 0, st, w.kinp.as<double>(), ld * nk, 1.0);
    for (int k = 0; k < nk; ++k)
      HIPCK(hipMemcpyAsync(w.kinp.as<double>() + (size_t)k * ld, pb->kp[k].d_kin.p, sizeof(double) * pb->kp[k].npw,
                           hipMemcpyDeviceToDevice, st));
    w.ld = ld;
    w.qcap = 0;
  }
  for (DevMem* m : {&w.C, &w.E, &w.Rj, &w.Tmp}) m->ensure(sizeof(CT) * sF * nk);
  w.s.ensure(sizeof(double) * nk * p);
  w.alpha.ensure(sizeof(double) * nk * p);
  w.Gm64.ensure(sizeof(z64) * pp * nk);
  w.PU64.ensure(sizeof(z64) * pp * nk);
  w.PU.ensure(sizeof(CT) * pp * nk);
  w.piv.ensure(sizeof(int) * p * nk);
  w.rank.ensure(sizeof(int) * nk);
  w.kmap.ensure(sizeof(int) * nk);
  w.live.ensure(sizeof(int) * nk);
  w.norms.ensure(sizeof(double) * p * nk);
  w.hstage.ensure(sizeof(int) * 3 * nk);
  w.done.ensure(sizeof(int) * nk);
  w.Xt.ensure(sizeof(CT) * (size_t)pb->nmax * p);
  b.grow(4 * p, 0);
  const KDesc* kd = pb->d_kdesc.as<KDesc>();
  CT* C = w.C.as<CT>();
  CT* E = w.E.as<CT>();
  CT* Rj = w.Rj.as<CT>();
  double* s = w.s.as<double>();
  double* alpha = w.alpha.as<double>();
  // C = Phi - (H X0 - X0 Sigma) with X0 = Phi / mu equals -R / mu
  hipLaunchKernelGGL(k_frame_to_pad<T>, dim3(nblk(sF), nk), dim3(256), 0, st, p, kd, R, -1.0 / mu, C, ld);
  HIPCK(hipGetLastError());
  const std::vector<double> nC2 = b.norms(C);
  // Sigma = Lambda - mu I in the eigenbasis of Lambda: s = w - mu, the same U
  affine(st, nk * p, lw, -mu, 1.0, s);
  // TPA: alpha_j = sum_G |k+G|^2/2 |phi_jG|^2
  frame_col_wnorm2(st, kd, nk, p, Phi, 1, alpha);
  // V_1 = rrqr(P^-1 C), W_1 = H V_1, A_1 = V_1^H W_1, C_1 = V_1^H C
  hipLaunchKernelGGL(k_tpa_pad<T>, dim3(nblk(sF), nk), dim3(256), 0, st, p, ld, w.kinp.as<double>(), alpha, C, Rj);
  HIPCK(hipGetLastError());
  std::vector<int> rk = b.rrqr(Rj, b.V(), b.sV(), rank_tol);
  std::vector<int> qeff(rk), live(nk, 1), act;
  for (int k = 0; k < nk; ++k) {
    if (rk[k] > 0) {
      act.push_back(k);
      continue;
    }
    // nothing to solve: X = X0
    live[k] = 0;
    const auto& K = pb->kp[k];
    axpby<double>(st, K.npw * p, 1.0 / mu, Phi + (int64_t)p * K.off, 0.0, X + (int64_t)p * K.off);
    info[k].relres = nC2[k] > 0 ? 1.0 : 0.0;
  }
  b.apply_H(0, act);
  int q = p;
  b.gram(q, q, b.V(), b.sV(), b.W(), b.sV(), b.A(), b.qcap(), (int64_t)b.qcap() * b.qcap());
  b.gram(q, p, b.V(), b.sV(), C, sF, b.Cj(), b.qcap(), (int64_t)b.qcap() * p);
  hipLaunchKernelGGL(k_fix_deflated, dim3(nk), dim3(64), 0, st, 0, p, w.rank.as<int>(), b.A(), (int64_t)b.qcap(),
                     (int64_t)b.qcap() * b.qcap(), big);
  int it = 0;
  for (;;) {
    if (act.empty()) break;
    ++it;
    const int qc = b.qcap();
    const int64_t sA = (int64_t)qc * qc, qp = (int64_t)q * p;
    // ---- projected A_q Y - Y Sigma = C_q per k (FP64), in the eigenbasis of
    // Sigma (the right-hand sides C_q U): up to kTriMax through one tridiagonal
    // reduction of A_q per k and a shifted tridiagonal solve per column, all
    // k-points in the same launches; beyond, through A_q = Q diag(wA) Q^H,
    // where every column is a diagonal division
    if (q > kTriMax) {
      w.wA.ensure(sizeof(double) * q * nk);
      w.QA.ensure(sizeof(z64) * (size_t)q * q * nk);
    }
    for (DevMem* m : {&w.T2, &w.Ct, &w.Y, &w.YS}) m->ensure(sizeof(z64) * qp * nk);
    z64* T2 = w.T2.as<z64>();
    z64* Ct = w.Ct.as<z64>();
    z64* Y = w.Y.as<z64>();
    z64* YS = w.YS.as<z64>();
    gemm_nn<double>(st, q, p, p, b.Cj(), qc, lU, p, 0, T2, q, 1.0, 0.0, 0.0, nk, (int64_t)qc * p, pp, qp);
    if (q <= kTriMax) {
      sylvester_tridiag_batched(st, q, p, nk, b.A(), qc, sA, s, T2, w.tri);
    } else {
      heev(st, q, b.A(), qc, sA, w.wA.as<double>(), q, w.QA.as<z64>(), q, (int64_t)q * q, nk,
           pb->d_info.as<int>(), w.eig);
      gemm_hn<double>(st, q, q, p, w.QA.as<z64>(), q, T2, q, Ct, q, 1.0, 0.0, pb->ws.gemm_part, nk, (int64_t)q * q,
                      qp, qp);
      hipLaunchKernelGGL(k_sylv_divide_b, dim3(nblk(qp), nk), dim3(256), 0, st, q, p, w.wA.as<double>(), (int64_t)q,
                         s, Ct, qp);
      gemm_nn<double>(st, q, q, p, w.QA.as<z64>(), q, Ct, q, 0, T2, q, 1.0, 0.0, 0.0, nk, (int64_t)q * q, qp, qp);
    }
    gemm_nn<double>(st, q, p, p, T2, q, lU, p, 1, Y, q, 1.0, 0.0, 0.0, nk, qp, pp, qp);
    hipLaunchKernelGGL(k_scale_cols_b, dim3(nblk(qp), nk), dim3(256), 0, st, q, p, s, T2);
    gemm_nn<double>(st, q, p, p, T2, q, lU, p, 1, YS, q, 1.0, 0.0, 0.0, nk, qp, pp, qp);
    HIPCK(hipGetLastError());
    const CT* Yt;
    const CT* Ys;
    if constexpr (sizeof(T) == 8) {
      Yt = Y;
      Ys = YS;
    } else {
      w.YT.ensure(sizeof(CT) * qp * nk);
      w.YST.ensure(sizeof(CT) * qp * nk);
      conv_b(st, q, p, Y, q, qp, w.YT.as<CT>(), q, qp, nk);
      conv_b(st, q, p, YS, q, qp, w.YST.as<CT>(), q, qp, nk);
      Yt = w.YT.as<CT>();
      Ys = w.YST.as<CT>();
    }
    // ---- E = C - (W Y - V Y Sigma)
    HIPCK(hipMemcpyAsync(E, C, sizeof(CT) * sF * nk, hipMemcpyDeviceToDevice, st));
    gemm_nn<T>(st, ld, q, p, b.W(), ld, Yt, q, 0, E, ld, -1.0, 0.0, 1.0, nk, b.sV(), qp, sF);
    gemm_nn<T>(st, ld, q, p, b.V(), ld, Ys, q, 0, E, ld, 1.0, 0.0, 1.0, nk, b.sV(), qp, sF);
    const std::vector<double> nE2 = b.norms(E);
    std::vector<int> still, done;
    for (int k : act) {
      const double relres = nC2[k] > 0 ? std::sqrt(nE2[k] / nC2[k]) : 0.0;
      if (!std::isfinite(relres)) fail(EAHP_ENONFINITE, "non-finite residual in the metric solve");
      if (relres <= rtol || it >= maxit) done.push_back(k);
    }
    if (done.size() > 1) {
      // X_k = X0 + V_k Y_k of every k-point that stops here: V Y for all
      // k-points in one product (the same sums per element as one k-point's
      // product), then one launch over the stopped ones
      w.XP.ensure(sizeof(CT) * sF * nk);
      gemm_nn<T>(st, ld, q, p, b.V(), ld, Yt, q, 0, w.XP.as<CT>(), ld, 1.0, 0.0, 0.0, nk, b.sV(), qp, sF);
      b.upload(w.done, done, 2);
      hipLaunchKernelGGL(k_pad_to_frame_x<T>, dim3(nblk((int64_t)pb->nmax * p), (unsigned)done.size()), dim3(256), 0,
                         st, p, kd, w.done.as<int>(), w.XP.as<CT>(), ld, sF, Phi, 1.0 / mu, X);
      HIPCK(hipGetLastError());
    }
    for (int k : act) {
      const double relres = nC2[k] > 0 ? std::sqrt(nE2[k] / nC2[k]) : 0.0;
      if (relres <= rtol || it >= maxit) {
        if (done.size() > 1) {
          info[k].iters = it;
          info[k].relres = relres;
          info[k].q = qeff[k];
          pb->fom_iters += it;
          live[k] = 0;
          continue;
        }
        // X_k = X0 + V_k Y_k, from this iteration's projected solution
        const auto& K = pb->kp[k];
        z64* Xk = X + (int64_t)p * K.off;
        axpby<double>(st, K.npw * p, 1.0 / mu, Phi + (int64_t)p * K.off, 0.0, Xk);
        if constexpr (sizeof(T) == 8) {
          gemm_nn<double>(st, K.npw, q, p, b.V() + k * b.sV(), ld, Y + k * qp, q, 0, Xk, K.npw, 1.0, 0.0, 1.0);
        } else {
          gemm_nn<float>(st, K.npw, q, p, b.V() + k * b.sV(), ld, Yt + k * qp, q, 0, w.Xt.as<CT>(), K.npw, 1.0, 0.0,
                         0.0);
          axpy_mixed(st, K.npw * p, 1.0, w.Xt.as<c32>(), Xk);
        }
        info[k].iters = it;
        info[k].relres = relres;
        info[k].q = qeff[k];
        pb->fom_iters += it;
        live[k] = 0;
      } else {
        still.push_back(k);
      }
    }
    act.swap(still);
    if (act.empty()) break;
    // ---- R_j = (I - V V^H) P^-1 E_j, projected twice (stopped k-points: zero)
    hipLaunchKernelGGL(k_tpa_pad<T>, dim3(nblk(sF), nk), dim3(256), 0, st, p, ld, w.kinp.as<double>(), alpha, E, Rj);
    b.upload(w.live, live, 0);
    hipLaunchKernelGGL(k_mask_blocks<T>, dim3(nblk(sF), nk), dim3(256), 0, st, sF, w.live.as<int>(), Rj, sF);
    HIPCK(hipGetLastError());
    w.T1.ensure(sizeof(CT) * qp * nk);
    for (int pass = 0; pass < 2; ++pass) {
      gemm_hn<T>(st, ld, q, p, b.V(), ld, Rj, ld, w.T1.as<CT>(), q, 1.0, 0.0, pb->ws.gemm_part, nk, b.sV(), sF, qp);
      gemm_nn<T>(st, ld, q, p, b.V(), ld, w.T1.as<CT>(), q, 0, Rj, ld, -1.0, 0.0, 1.0, nk, b.sV(), qp, sF);
    }
    b.grow(q + p, q);
    const int qc2 = b.qcap();
    CT* Vn = b.V() + (int64_t)q * ld;
    rk = b.rrqr(Rj, Vn, b.sV(), rank_tol);
    std::vector<int> hv;
    for (int k : act) {
      qeff[k] += rk[k];
      if (rk[k] > 0) hv.push_back(k);
    }
    b.apply_H(q, hv);
    // border A with V^H W_new (rows 0..q+p) and mirror; C_{j+1} = [C_j ; V_new^H C]
    b.gram(q + p, p, b.V(), b.sV(), b.W() + (int64_t)q * ld, b.sV(), b.A() + (int64_t)q * qc2, qc2,
           (int64_t)qc2 * qc2);
    hipLaunchKernelGGL(k_border_mirror_b, dim3(nblk((int64_t)q * p), nk), dim3(256), 0, st, q, p, b.A(),
                       (int64_t)qc2, (int64_t)qc2 * qc2);
    b.gram(p, p, Vn, b.sV(), C, sF, b.Cj() + q, qc2, (int64_t)qc2 * p);
    hipLaunchKernelGGL(k_fix_deflated, dim3(nk), dim3(64), 0, st, q, p, w.rank.as<int>(), b.A(), (int64_t)qc2,
                       (int64_t)qc2 * qc2, big);
    HIPCK(hipGetLastError());
    q += p;
  }
}

template void fom_batch<double>(eahp_problem*, const z64*, const z64*, const double*, const z64*, double, double, int,
                                double, z64*, std::vector<FomInfo>&);
template void fom_batch<float>(eahp_problem*, const z64*, const z64*, const double*, const z64*, double, double, int,
                               double, z64*, std::vector<FomInfo>&);

}  // namespace eahp
