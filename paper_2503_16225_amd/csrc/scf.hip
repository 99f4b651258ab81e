// Self-consistent field iteration, the method the paper compares EARCG with
// and uses to make its initial guesses (Sec. 5.2): at the potential of the
// current density, the p lowest eigenpairs of every H_k by a block
// preconditioned eigensolver; the output density; Anderson mixing of the
// density (the nonlinear eigenvector problem of eq. (1.3) with the Aufbau
// principle, Sec. 2.1).
//
// Eigensolver: LOBPCG on the basis [X, W, P] per k-point.  X holds the Ritz
// vectors, W the TPA-preconditioned residuals (alpha_j = the kinetic energy
// of x_j, as in the metric solve), P the previous update directions.  W and P
// are orthogonalised against X (and W against P) twice and orthonormalised by
// a pivoted Cholesky QR, taken twice; directions whose remaining norm falls
// below 1e-7 of the largest are dropped, which also stops refining converged
// bands.  H P is carried along through the same transformations, so an
// iteration applies H only to W.  The Rayleigh-Ritz problem on the compact
// basis is a Hermitian eigenproblem of order p + r_W + r_P.
//
// Mixing: with history x_i = rho_in, f_i = rho_out - rho_in (at most `depth`
// entries), dX and dF the differences of consecutive entries, g the least-
// squares solution of dF g = f (modified Gram-Schmidt QR of dF, columns with
// r_jj <= 1e-13 max r dropped), rho_next = rho - dX g + beta (f - dF g);
// without history rho_next = rho + beta f.  Stop when
// ||rho_out - rho_in||_2 (the L2 norm over the cell) <= tol, with the
// adaptive eigensolver tolerance (0.1 x the last residual, within [1e-12,
// 1e-2]) only after a step solved to at most max(1e-12, 0.1 tol).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "devcommon.h"
#include "ops.h"

namespace eahp {

namespace {

// R[:, j] = HX[:, j] - theta_j X[:, j]
__global__ void k_resid_diag(int64_t n, int p, const z64* __restrict__ X, const z64* __restrict__ HX,
                             const double* __restrict__ th, z64* __restrict__ R) {
  const int64_t tot = n * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const double t = th[e / n];
    R[e] = mk<double>(HX[e].x - t * X[e].x, HX[e].y - t * X[e].y);
  }
}

// C[:, j] = V[:, idx[j]] (m rows)
__global__ void k_gather_cols(int m, int p, const z64* __restrict__ V, int ldv, const int* __restrict__ idx,
                              z64* __restrict__ C) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * p; e += gridDim.x * blockDim.x) {
    const int j = e / m, i = e - j * m;
    C[e] = V[i + (int64_t)idx[j] * ldv];
  }
}

__global__ void k_zero_cols(int64_t n, int c0, int c1, z64* __restrict__ A) {
  const int64_t tot = n * (c1 - c0);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x)
    A[c0 * n + e] = mk<double>(0, 0);
}

// partial real dot products of the pairs (x_a, y_a), a < npair, over n: one
// row of 256 partials per pair, summed in a fixed order by k_dot_final
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, int npair, const double* const* __restrict__ xs,
                                                     const double* const* __restrict__ ys, double* __restrict__ part) {
  __shared__ double red[256];
  const int a = blockIdx.y;
  const double* x = xs[a];
  const double* y = ys[a];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[a * gridDim.x + blockIdx.x] = red[0];
}
__global__ void k_dot_final(int npair, int nb, const double* __restrict__ part, double* __restrict__ out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= npair) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[a * nb + b];
  out[a] = s;
}

// y = sum_a c_a x_a + d z over n (up to 32 terms)
struct LinComb {
  int nt;
  const double* x[32];
  double c[32];
};
__global__ void k_lincomb(int64_t n, LinComb L, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int a = 0; a < L.nt; ++a) s += L.c[a] * L.x[a][i];
    y[i] = s;
  }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

void LobWork::ensure(int64_t n_, int p_) {
  const size_t f = sizeof(z64) * (size_t)n_ * p_;
  S.ensure(3 * f);
  HS.ensure(3 * f);
  T1.ensure(f);
  T2.ensure(f);
  T3.ensure(f);
  T4.ensure(f);
  R.ensure(f);
  const size_t m = 3 * (size_t)p_;
  A.ensure(sizeof(z64) * m * m);
  V.ensure(sizeof(z64) * m * m);
  w.ensure(sizeof(double) * m);
  C.ensure(sizeof(z64) * m * p_);
  Y.ensure(sizeof(z64) * m * m);
  G.ensure(sizeof(z64) * m * m);
  PU.ensure(sizeof(z64) * m * m);
  piv.ensure(sizeof(int) * m);
  th.ensure(sizeof(double) * p_);
  rn.ensure(sizeof(double) * p_);
  alpha.ensure(sizeof(double) * p_);
  idx.ensure(sizeof(int) * p_);
}

namespace {

int read_rank(eahp_problem* pb) {
  hipStream_t st = pb->ctx->stream;
  HIPCK(hipMemcpyAsync(pb->h_info, pb->d_info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return pb->h_info[0];
}

// Orthonormal basis of the c columns of A (n x c, ld n) in place by pivoted
// Cholesky QR taken twice, the same column transformations applied to HA
// (when given); columns beyond the rank are zeroed.  Returns the rank.
int cholqr_pair(eahp_problem* pb, int64_t n, int c, z64* A, z64* HA, double tol, LobWork& w) {
  hipStream_t st = pb->ctx->stream;
  if (c <= 0) return 0;
  int cols = c;
  for (int pass = 0; pass < 2 && cols > 0; ++pass) {
    gemm_hn<double>(st, n, cols, cols, A, n, A, n, w.G.as<z64>(), cols, 1.0, 0.0, pb->ws.gemm_part);
    pchol_inv(st, cols, w.G.as<z64>(), cols, pass == 0 ? tol : 0.0, w.piv.as<int>(), pb->d_info.as<int>(),
              w.PU.as<z64>(), cols, nullptr, pb->ws.chol);
    const int r = std::max(0, read_rank(pb));
    if (r > 0) {
      gemm_nn<double>(st, n, cols, r, A, n, w.PU.as<z64>(), cols, 0, w.T4.as<z64>(), n, 1.0, 0.0, 0.0);
      HIPCK(hipMemcpyAsync(A, w.T4.p, sizeof(z64) * n * r, hipMemcpyDeviceToDevice, st));
      if (HA) {
        gemm_nn<double>(st, n, cols, r, HA, n, w.PU.as<z64>(), cols, 0, w.T4.as<z64>(), n, 1.0, 0.0, 0.0);
        HIPCK(hipMemcpyAsync(HA, w.T4.p, sizeof(z64) * n * r, hipMemcpyDeviceToDevice, st));
      }
    }
    cols = r;
  }
  if (cols < c) {
    hipLaunchKernelGGL(k_zero_cols, dim3(grid_for(n * (c - cols))), dim3(256), 0, st, n, cols, c, A);
    if (HA) hipLaunchKernelGGL(k_zero_cols, dim3(grid_for(n * (c - cols))), dim3(256), 0, st, n, cols, c, HA);
    HIPCK(hipGetLastError());
  }
  return cols;
}

// B -= A (A^H B), and HB -= HA (A^H B) when given (A n x a orthonormal, B n x b).
void project_out(eahp_problem* pb, int64_t n, int a, const z64* A, const z64* HA, int b, z64* B, z64* HB,
                 LobWork& w) {
  if (a <= 0 || b <= 0) return;
  hipStream_t st = pb->ctx->stream;
  gemm_hn<double>(st, n, a, b, A, n, B, n, w.Y.as<z64>(), a, 1.0, 0.0, pb->ws.gemm_part);
  gemm_nn<double>(st, n, a, b, A, n, w.Y.as<z64>(), a, 0, B, n, -1.0, 0.0, 1.0);
  if (HB) gemm_nn<double>(st, n, a, b, HA, n, w.Y.as<z64>(), a, 0, HB, n, -1.0, 0.0, 1.0);
}

// Eigenpairs of the Hermitian m x m matrix in w.A: the p lowest, ascending;
// eigenvectors into w.C (m x p), values into theta (host) and w.th (device).
void lowest_eigenpairs(eahp_problem* pb, int m, int p, double* theta, LobWork& w) {
  hipStream_t st = pb->ctx->stream;
  hermitize(st, m, w.A.as<z64>(), m, 0, 1);
  heev(st, m, w.A.as<z64>(), m, 0, w.w.as<double>(), 0, w.V.as<z64>(), m, 0, 1, pb->d_info.as<int>(), pb->ws.eig);
  std::vector<double> ev(m);
  HIPCK(hipMemcpyAsync(ev.data(), w.w.p, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (double v : ev)
    if (!std::isfinite(v)) fail(EAHP_ENONFINITE, "non-finite Ritz value");
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ev[a] < ev[b]; });
  order.resize(p);
  for (int j = 0; j < p; ++j) theta[j] = ev[order[j]];
  HIPCK(hipMemcpyAsync(w.idx.p, order.data(), sizeof(int) * p, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(w.th.p, theta, sizeof(double) * p, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for((int64_t)m * p)), dim3(256), 0, st, m, p, w.V.as<z64>(), m,
                     w.idx.as<int>(), w.C.as<z64>());
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));  // theta and order live on this host stack frame
}

}  // namespace

// LOBPCG for the p lowest eigenpairs of H_k at the current potential.  X
// (n_k x p, ld n_k) holds the start block on entry and the Ritz vectors on
// return; theta (host, p) the Ritz values; rnorm_max the largest residual
// norm.  Returns the iterations done.
int lobpcg_k(eahp_problem* pb, int ik, z64* X, double tol, int maxit, double* theta, double* rnorm_max,
             int64_t* napply) {
  hipStream_t st = pb->ctx->stream;
  LobWork& w = pb->arena->lob;
  const int p = pb->p;
  auto& K = pb->kp[ik];
  const int64_t n = K.npw;
  if (n < 3 * p) fail(EAHP_EINVAL, "fewer plane waves than 3 p at a k-point");
  w.ensure(n, p);
  z64* S = w.S.as<z64>();
  z64* HS = w.HS.as<z64>();
  z64* Xs = S;
  z64* Ws = S + n * p;
  z64* Ps = S + 2 * n * p;
  z64* HXs = HS;
  z64* HWs = HS + n * p;
  z64* HPs = HS + 2 * n * p;
  HIPCK(hipMemcpyAsync(Xs, X, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
  if (cholqr_pair(pb, n, p, Xs, nullptr, 1e-14, w) < p) fail(EAHP_EINVAL, "start block of the eigensolver is rank deficient");
  apply_H_block<double>(pb, ik, p, Xs, HXs);
  *napply += p;
  gemm_hn<double>(st, n, p, p, Xs, n, HXs, n, w.A.as<z64>(), p, 1.0, 0.0, pb->ws.gemm_part);
  lowest_eigenpairs(pb, p, p, theta, w);
  gemm_nn<double>(st, n, p, p, Xs, n, w.C.as<z64>(), p, 0, w.T1.as<z64>(), n, 1.0, 0.0, 0.0);
  gemm_nn<double>(st, n, p, p, HXs, n, w.C.as<z64>(), p, 0, w.T2.as<z64>(), n, 1.0, 0.0, 0.0);
  HIPCK(hipMemcpyAsync(Xs, w.T1.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
  HIPCK(hipMemcpyAsync(HXs, w.T2.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
  int rP = 0;
  int it = 0;
  std::vector<double> rn(p);
  for (;; ++it) {
    hipLaunchKernelGGL(k_resid_diag, dim3(grid_for(n * p)), dim3(256), 0, st, n, p, Xs, HXs, w.th.as<double>(),
                       w.R.as<z64>());
    HIPCK(hipGetLastError());
    col_weighted_norm2(st, n, p, w.R.as<z64>(), n, nullptr, w.rn.as<double>());
    HIPCK(hipMemcpyAsync(rn.data(), w.rn.p, sizeof(double) * p, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    double rmax = 0.0;
    for (double v : rn) rmax = std::max(rmax, std::sqrt(std::max(v, 0.0)));
    if (!std::isfinite(rmax)) fail(EAHP_ENONFINITE, "non-finite eigensolver residual");
    *rnorm_max = rmax;
    if (rmax <= tol || it >= maxit) break;
    // W: preconditioned residuals, orthogonalised against X and P, orthonormalised
    col_weighted_norm2(st, n, p, Xs, n, K.d_kin.as<double>(), w.alpha.as<double>());
    tpa_apply<double>(st, n, p, K.d_kin.as<double>(), w.alpha.as<double>(), w.R.as<z64>(), n, Ws, n);
    for (int pass = 0; pass < 2; ++pass) {
      project_out(pb, n, p, Xs, nullptr, p, Ws, nullptr, w);
      project_out(pb, n, rP, Ps, nullptr, p, Ws, nullptr, w);
    }
    const int rW = cholqr_pair(pb, n, p, Ws, nullptr, 1e-14, w);
    if (rW > 0) {
      apply_H_block<double>(pb, ik, rW, Ws, HWs);
      *napply += rW;
    }
    // Rayleigh-Ritz on [X, W(:, :rW), P(:, :rP)]
    const int m = p + rW + rP;
    const int off[3] = {0, p, p + rW}, len[3] = {p, rW, rP};
    const z64* blk[3] = {Xs, Ws, Ps};
    const z64* hblk[3] = {HXs, HWs, HPs};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        if (len[a] > 0 && len[b] > 0)
          gemm_hn<double>(st, n, len[a], len[b], blk[a], n, hblk[b], n, w.A.as<z64>() + off[a] + (int64_t)off[b] * m,
                          m, 1.0, 0.0, pb->ws.gemm_part);
    lowest_eigenpairs(pb, m, p, theta, w);
    const z64* Cm = w.C.as<z64>();
    // X+ = X C_X + W C_W + P C_P, P+ = W C_W + P C_P, and the same for H
    gemm_nn<double>(st, n, p, p, Xs, n, Cm, m, 0, w.T1.as<z64>(), n, 1.0, 0.0, 0.0);
    gemm_nn<double>(st, n, p, p, HXs, n, Cm, m, 0, w.T2.as<z64>(), n, 1.0, 0.0, 0.0);
    bool first = true;
    for (int a = 1; a < 3; ++a) {
      if (len[a] == 0) continue;
      gemm_nn<double>(st, n, len[a], p, blk[a], n, Cm + off[a], m, 0, w.T3.as<z64>(), n, 1.0, 0.0, first ? 0.0 : 1.0);
      gemm_nn<double>(st, n, len[a], p, hblk[a], n, Cm + off[a], m, 0, w.R.as<z64>(), n, 1.0, 0.0,
                      first ? 0.0 : 1.0);
      first = false;
    }
    if (!first) {  // X+ = X C_X + P+, H X+ = H X C_X + H P+
      axpby<double>(st, n * p, 1.0, w.T3.as<z64>(), 1.0, w.T1.as<z64>());
      axpby<double>(st, n * p, 1.0, w.R.as<z64>(), 1.0, w.T2.as<z64>());
    }
    HIPCK(hipMemcpyAsync(Xs, w.T1.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpyAsync(HXs, w.T2.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
    if (first) {
      rP = 0;
      continue;
    }
    HIPCK(hipMemcpyAsync(Ps, w.T3.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpyAsync(HPs, w.R.p, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
    for (int pass = 0; pass < 2; ++pass) project_out(pb, n, p, Xs, HXs, p, Ps, HPs, w);
    rP = cholqr_pair(pb, n, p, Ps, HPs, 1e-14, w);
  }
  HIPCK(hipMemcpyAsync(X, Xs, sizeof(z64) * n * p, hipMemcpyDeviceToDevice, st));
  return it;
}

// ---------------------------------------------------------------- SCF
namespace {

// real dot products <x_a, y_a> over n doubles, returned on the host
void dots(eahp_problem* pb, int64_t n, const std::vector<std::pair<const double*, const double*>>& pairs,
          std::vector<double>& out) {
  hipStream_t st = pb->ctx->stream;
  const int np = (int)pairs.size();
  out.assign(np, 0.0);
  if (np == 0) return;
  const int nb = 256;
  std::vector<const double*> xs(np), ys(np);
  for (int a = 0; a < np; ++a) {
    xs[a] = pairs[a].first;
    ys[a] = pairs[a].second;
  }
  pb->ws.small.ensure(sizeof(void*) * 2 * np);
  const double** dxy = pb->ws.small.as<const double*>();
  HIPCK(hipMemcpyAsync(dxy, xs.data(), sizeof(void*) * np, hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(dxy + np, ys.data(), sizeof(void*) * np, hipMemcpyHostToDevice, st));
  pb->ws.partial.ensure(sizeof(double) * ((size_t)nb * np + np));
  double* part = pb->ws.partial.as<double>();
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, np), dim3(256), 0, st, n, np, dxy, dxy + np, part);
  hipLaunchKernelGGL(k_dot_final, dim3((np + 63) / 64), dim3(64), 0, st, np, nb, part, part + (size_t)nb * np);
  HIPCK(hipGetLastError());
  HIPCK(hipMemcpyAsync(out.data(), part + (size_t)nb * np, sizeof(double) * np, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
}

void lincomb(eahp_problem* pb, int64_t n, const std::vector<std::pair<double, const double*>>& terms, double* y) {
  LinComb L{};
  if (terms.size() > 32) fail(EAHP_EINVAL, "too many terms");
  L.nt = (int)terms.size();
  for (int a = 0; a < L.nt; ++a) {
    L.c[a] = terms[a].first;
    L.x[a] = terms[a].second;
  }
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, pb->ctx->stream, n, L, y);
  HIPCK(hipGetLastError());
}

}  // namespace

void scf_run(eahp_problem* pb, z64* Psi, const eahp_scf_params& prm, eahp_scf_stats* out) {
  hipStream_t st = pb->ctx->stream;
  const auto t0 = std::chrono::steady_clock::now();
  if (!(prm.tol > 0) || prm.maxit < 0 || !(prm.beta > 0) || prm.depth < 1 || prm.depth > 16 || prm.eig_maxit < 1 ||
      prm.eig_tol < 0)
    fail(EAHP_EINVAL, "invalid SCF parameters");
  const int64_t Ng = pb->Ng;
  const int D = prm.depth;
  DevMem hx, hf, rin, qb;
  hx.alloc(sizeof(double) * Ng * D);
  hf.alloc(sizeof(double) * Ng * D);
  rin.alloc(sizeof(double) * Ng);
  qb.alloc(sizeof(double) * Ng * std::max(D - 1, 1));
  double* rho = pb->d_rho.as<double>();
  double* rhoin = rin.as<double>();
  const double l2 = std::sqrt(pb->Omega / (double)Ng);
  int64_t napply = 0;
  int eig_iters = 0;
  // the start block orthonormalised per k (its span is kept); rho_in of the
  // first step is its density
  for (int ik = 0; ik < pb->nk; ++ik) {
    auto& K = pb->kp[ik];
    if (K.npw < 3 * (int64_t)pb->p) fail(EAHP_EINVAL, "fewer plane waves than 3 p at a k-point");
    pb->arena->lob.ensure(K.npw, pb->p);
    if (cholqr_pair(pb, K.npw, pb->p, Psi + (int64_t)pb->p * K.off, nullptr, 1e-14, pb->arena->lob) < pb->p)
      fail(EAHP_EINVAL, "start block is rank deficient");
  }
  density_potentials(pb, Psi);
  HIPCK(hipMemcpyAsync(rhoin, rho, sizeof(double) * Ng, hipMemcpyDeviceToDevice, st));
  std::vector<double> theta(pb->p);
  int nh = 0, head = 0;  // history entries, next slot
  double res = INFINITY, eig_tol = prm.eig_tol > 0 ? prm.eig_tol : 1e-2;
  int it = 0;
  for (;; ++it) {
    // eigenpairs at V_eff(rho_in), warm-started from the previous block
    for (int ik = 0; ik < pb->nk; ++ik) {
      double rmax = 0;
      eig_iters += lobpcg_k(pb, ik, Psi + (int64_t)pb->p * pb->kp[ik].off, eig_tol, prm.eig_maxit, theta.data(),
                            &rmax, &napply);
    }
    density_potentials(pb, Psi);  // rho_out (and its potential, replaced below)
    // f = rho_out - rho_in into the history slot, x = rho_in
    double* xs = hx.as<double>() + (int64_t)head * Ng;
    double* fs = hf.as<double>() + (int64_t)head * Ng;
    HIPCK(hipMemcpyAsync(xs, rhoin, sizeof(double) * Ng, hipMemcpyDeviceToDevice, st));
    lincomb(pb, Ng, {{1.0, rho}, {-1.0, rhoin}}, fs);
    std::vector<double> d;
    dots(pb, Ng, {{fs, fs}}, d);
    res = std::sqrt(std::max(d[0], 0.0)) * l2;
    if (!std::isfinite(res)) fail(EAHP_ENONFINITE, "non-finite density residual");
    // with the adaptive eigensolver tolerance a small residual is accepted only
    // from a step whose eigenpairs were solved to 0.1 tol (a loose solve from a
    // nearly converged block returns it unchanged, and rho_out = rho_in)
    const double eig_need = std::max(1e-12, 0.1 * prm.tol);
    const bool solved_enough = prm.eig_tol > 0 || eig_tol <= eig_need * (1.0 + 1e-12);
    if ((res <= prm.tol && solved_enough) || it >= prm.maxit) break;
    if (prm.eig_tol <= 0) eig_tol = std::min(1e-2, std::max(1e-12, 0.1 * std::max(res, prm.tol)));
    nh = std::min(nh + 1, D);
    // entries oldest -> newest
    std::vector<const double*> X_(nh), F_(nh);
    for (int i = 0; i < nh; ++i) {
      const int slot = (head - (nh - 1) + i + D) % D;
      X_[i] = hx.as<double>() + (int64_t)slot * Ng;
      F_[i] = hf.as<double>() + (int64_t)slot * Ng;
    }
    head = (head + 1) % D;
    std::vector<std::pair<double, const double*>> terms;
    if (nh >= 2) {
      // least squares dF g = f by modified Gram-Schmidt on the columns dF_i = F_{i+1} - F_i
      const int m = nh - 1;
      double* Q = qb.as<double>();
      std::vector<double> Rm((size_t)m * m, 0.0), rdiag(m, 0.0);
      std::vector<int> keep;
      for (int j = 0; j < m; ++j) {
        double* qj = Q + (int64_t)j * Ng;
        lincomb(pb, Ng, {{1.0, F_[j + 1]}, {-1.0, F_[j]}}, qj);
        for (int i : keep) {
          dots(pb, Ng, {{Q + (int64_t)i * Ng, qj}}, d);
          Rm[i + (size_t)j * m] = d[0];
          lincomb(pb, Ng, {{1.0, qj}, {-d[0], Q + (int64_t)i * Ng}}, qj);
        }
        dots(pb, Ng, {{qj, qj}}, d);
        const double r = std::sqrt(std::max(d[0], 0.0));
        double rmax = r;
        for (int i : keep) rmax = std::max(rmax, rdiag[i]);
        if (r <= 1e-13 * rmax || r == 0.0) continue;  // dependent column: its coefficient stays 0
        rdiag[j] = r;
        Rm[j + (size_t)j * m] = r;
        lincomb(pb, Ng, {{1.0 / r, qj}}, qj);
        keep.push_back(j);
      }
      // g = R^-1 Q^T f over the kept columns (back substitution)
      std::vector<std::pair<const double*, const double*>> pr;
      for (int i : keep) pr.push_back({Q + (int64_t)i * Ng, fs});
      dots(pb, Ng, pr, d);
      std::vector<double> qf(m, 0.0), g(m, 0.0);
      for (size_t a = 0; a < keep.size(); ++a) qf[keep[a]] = d[a];
      for (int a = (int)keep.size() - 1; a >= 0; --a) {
        const int j = keep[a];
        double s = qf[j];
        for (size_t b = a + 1; b < keep.size(); ++b) s -= Rm[j + (size_t)keep[b] * m] * g[keep[b]];
        g[j] = s / Rm[j + (size_t)j * m];
      }
      // rho_next = x - dX g + beta (f - dF g), dX_i = X_{i+1} - X_i, x = X_m, f = F_m:
      // the coefficient of X_j is g_j - g_{j-1} (+1 for j = m), that of F_j beta times it
      for (int j = 0; j <= m; ++j) {
        const double c = (j < m ? g[j] : 0.0) - (j >= 1 ? g[j - 1] : 0.0) + (j == m ? 1.0 : 0.0);
        if (c == 0.0) continue;
        terms.push_back({c, X_[j]});
        terms.push_back({prm.beta * c, F_[j]});
      }
    } else {
      terms.push_back({1.0, rhoin});
      terms.push_back({prm.beta, fs});
    }
    lincomb(pb, Ng, terms, rho);
    HIPCK(hipMemcpyAsync(rhoin, rho, sizeof(double) * Ng, hipMemcpyDeviceToDevice, st));
    potentials(pb);
  }
  PointScalars ps;
  evaluate_energy(pb, Psi, &ps);
  HIPCK(hipStreamSynchronize(st));
  if (out) {
    out->iters = it + 1;
    out->napply = napply;
    out->eig_iters = eig_iters;
    out->energy = ps.E;
    out->res = res;
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (res > prm.tol) fail(EAHP_ENOCONV, "SCF reached maxit above tolerance");
}

}  // namespace eahp
