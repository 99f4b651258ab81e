// Manifold operations on frames, per k-point: polar retraction (eqs. (3.1)-(3.2)),
// differentiated-retraction transports (Prop. 3.1 and its closed form for
// xi = tau eta, Sec. 3.2), the qR retraction and its differentiated transport, the energy-adaptive gradient (Sec. 5.2) and the
// preconditioned block FOM for the Sylvester equation (Appendix A, Algorithm 4).
#include <algorithm>
#include <cmath>

#include "ops.h"
#include "setup.h"

namespace eahp {



// ---------------------------------------------------------------- retraction
void retract(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, z64* out, RetractFactors& F) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  const int64_t N = pb->ntot * p;
  F.d.ensure(sizeof(double) * nk * p);
  F.V.ensure(sizeof(z64) * nk * pp);
  F.Sinv.ensure(sizeof(z64) * nk * pp);
  Scratch& s = pb->arena->s;
  s.a.ensure(sizeof(z64) * N);
  s.b.ensure(sizeof(z64) * nk * pp);
  z64* Psi = s.a.as<z64>();
  z64* Gm = s.b.as<z64>();
  axpby<double>(st, N, 1.0, Phi, 0.0, Psi);
  axpby<double>(st, N, tau, eta, 1.0, Psi);
  frames_hn(pb, Psi, Psi, Gm);
  heev(st, p, Gm, p, pp, F.d.as<double>(), p, F.V.as<z64>(), p, pp, nk, pb->d_info.as<int>(), pb->ws.eig);
  minval(st, nk * p, F.d.as<double>(), scal(pb, S_MIN));
  spectral_fn(st, p, F.V.as<z64>(), p, pp, F.d.as<double>(), p, -0.5, F.Sinv.as<z64>(), p, pp, nk);
  frames_nn(pb, Psi, F.Sinv.as<z64>(), 0, out, 1.0, 0.0);
  fetch_scalars(pb, S_MIN + 1);
  const double dmin = pb->h_scal[S_MIN];
  if (!std::isfinite(dmin)) fail(EAHP_ENONFINITE, "non-finite Gram matrix in the retraction");
  if (!(dmin > 0.0)) fail(EAHP_ENOTPD, "retraction Gram matrix not positive definite");
}

void line_prepare(eahp_problem* pb, const z64* Phi, const z64* eta, LineFactors& L) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  for (DevMem* m : {&L.E0, &L.A1, &L.V, &L.Dt, &L.T}) m->ensure(sizeof(z64) * nk * pp);
  L.w.ensure(sizeof(double) * nk * p);
  Scratch& s = pb->arena->s;
  s.b.ensure(sizeof(z64) * nk * pp);
  frames_hn(pb, Phi, Phi, L.E0.as<z64>());
  frames_hn(pb, Phi, eta, L.A1.as<z64>());
  frames_hn(pb, eta, eta, s.b.as<z64>());
  hermitize(st, p, L.E0.as<z64>(), p, pp, nk);
  add_diag(st, p, L.E0.as<z64>(), p, pp, -1.0, nk);
  hermitize(st, p, L.A1.as<z64>(), p, pp, nk);  // (X + X^H) / 2 with X = Phi^H eta
  heev(st, p, s.b.as<z64>(), p, pp, L.w.as<double>(), p, L.V.as<z64>(), p, pp, nk, pb->d_info.as<int>(), pb->ws.eig);
}

bool retract_line(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, LineFactors& L, z64* out,
                  RetractFactors& F) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  const int64_t N = pb->ntot * p;
  z64* Dt = L.Dt.as<z64>();
  z64* T = L.T.as<z64>();
  const z64* V = L.V.as<z64>();
  // Delta = E0 + 2 tau A1h
  axpby<double>(st, nk * pp, 2.0 * tau, L.A1.as<z64>(), 0.0, Dt);
  axpby<double>(st, nk * pp, 1.0, L.E0.as<z64>(), 1.0, Dt);
  dot_re(st, nk * pp, Dt, Dt, scal(pb, S_NRM2), pb->ws.partial);
  fetch_scalars(pb, S_NRM2 + 1);
  const double nd2 = pb->h_scal[S_NRM2];
  if (!std::isfinite(nd2)) fail(EAHP_ENONFINITE, "non-finite Gram matrix in the retraction");
  // second-order remainder below 1e-16 (d >= 1 bounds every divided difference)
  if (nd2 > 1e-16) return false;
  F.d.ensure(sizeof(double) * nk * p);
  F.V.ensure(sizeof(z64) * nk * pp);
  F.Sinv.ensure(sizeof(z64) * nk * pp);
  // Dt <- V^H Delta V
  gemm_hn<double>(st, p, p, p, V, p, Dt, p, T, p, 1.0, 0.0, pb->ws.gemm_part, nk, pp, pp, pp);
  gemm_nn<double>(st, p, p, p, T, p, V, p, 0, Dt, p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  polar_first_order(st, p, L.w.as<double>(), tau, Dt, F.d.as<double>(), T, nk);
  // Sinv = V Mt V^H
  gemm_nn<double>(st, p, p, p, V, p, T, p, 0, Dt, p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  gemm_nn<double>(st, p, p, p, Dt, p, V, p, 1, F.Sinv.as<z64>(), p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  hermitize(st, p, F.Sinv.as<z64>(), p, pp, nk);
  HIPCK(hipMemcpyAsync(F.V.p, V, sizeof(z64) * nk * pp, hipMemcpyDeviceToDevice, st));
  Scratch& s = pb->arena->s;
  s.a.ensure(sizeof(z64) * N);
  z64* Psi = s.a.as<z64>();
  axpby<double>(st, N, 1.0, Phi, 0.0, Psi);
  axpby<double>(st, N, tau, eta, 1.0, Psi);
  frames_nn(pb, Psi, F.Sinv.as<z64>(), 0, out, 1.0, 0.0);
  return true;
}

// ---------------------------------------------------------------- qR retraction
// qf(Phi + tau eta) = Psi R^-1 with Psi^H Psi = R^H R (R upper triangular with a
// positive diagonal), the Gram-Schmidt retraction the paper names as the
// alternative to the polar one (Sec. 3.1).  R^-1 per k goes to F.Sinv.
void retract_qr(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, z64* out, RetractFactors& F) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  const int64_t N = pb->ntot * p;
  F.Sinv.ensure(sizeof(z64) * nk * pp);
  Scratch& s = pb->arena->s;
  s.a.ensure(sizeof(z64) * N);
  s.b.ensure(sizeof(z64) * nk * pp);
  s.g.ensure(sizeof(int) * (size_t)nk * (p + 1));
  z64* Psi = s.a.as<z64>();
  z64* Gm = s.b.as<z64>();
  int* piv = s.g.as<int>();
  int* rank = pb->d_info.as<int>();
  if (nk > 1024) fail(EAHP_EINVAL, "too many k-points for the qR retraction");
  axpby<double>(st, N, 1.0, Phi, 0.0, Psi);
  axpby<double>(st, N, tau, eta, 1.0, Psi);
  frames_hn(pb, Psi, Psi, Gm);
  for (int ik = 0; ik < nk; ++ik)
    pchol_inv(st, p, Gm + ik * pp, p, 0.0, piv + (size_t)ik * p, rank + ik, F.Sinv.as<z64>() + ik * pp, p, nullptr,
              pb->ws.chol, false);
  frames_nn(pb, Psi, F.Sinv.as<z64>(), 0, out, 1.0, 0.0);
  HIPCK(hipMemcpyAsync(pb->h_info, rank, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (int ik = 0; ik < nk; ++ik)
    if (pb->h_info[ik] != p) fail(EAHP_ENOTPD, "retraction Gram matrix not positive definite");
}

// Differentiated qR retraction at the new point Q = qf(psi) with psi = Q R:
// with M = Q^H v R^-1, D qf(psi)[v] = v R^-1 + Q (Omega(M) - M), Omega(M) the
// skew-Hermitian part fixed by M's strictly lower triangle and the imaginary
// part of its diagonal.  Needs only F.Sinv = R^-1 of the retraction.
void transport_qr(eahp_problem* pb, const z64* Q, const z64* v, const RetractFactors& F, z64* out) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  Scratch& s = pb->arena->s;
  s.d.ensure(sizeof(z64) * nk * pp);
  s.e.ensure(sizeof(z64) * nk * pp);
  z64* W = s.d.as<z64>();
  z64* M = s.e.as<z64>();
  const z64* Rinv = F.Sinv.as<z64>();
  frames_hn(pb, Q, v, W);
  gemm_nn<double>(st, p, p, p, W, p, Rinv, p, 0, M, p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  qr_omega_minus(st, p, M, p, pp, W, p, pp, nk);  // W <- Omega(M) - M
  frames_nn(pb, v, Rinv, 0, out, 1.0, 0.0);
  frames_nn(pb, Q, W, 0, out, 1.0, 1.0);
}

void lambda_eig(eahp_problem* pb, const z64* Lam, LamEig& E) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  E.w.ensure(sizeof(double) * nk * p);
  E.U.ensure(sizeof(z64) * nk * pp);
  Scratch& s = pb->arena->s;
  s.b.ensure(sizeof(z64) * nk * pp);
  copy2d(st, p, p * nk, Lam, p, s.b.as<z64>(), p);
  heev(st, p, s.b.as<z64>(), p, pp, E.w.as<double>(), p, E.U.as<z64>(), p, pp, nk, pb->d_info.as<int>(), pb->ws.eig);
}

// ---------------------------------------------------------------- transports
// T(eta) = eta S^-1 - tau R(tau eta) (eta S^-1)^H (eta S^-1)
void transport_self(eahp_problem* pb, const z64* Phi_new, const z64* eta, double tau, const RetractFactors& F,
                    z64* out) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p;
  const int64_t pp = (int64_t)p * p;
  Scratch& s = pb->arena->s;
  s.c.ensure(sizeof(z64) * pb->ntot * p);
  s.d.ensure(sizeof(z64) * pb->nk * pp);
  z64* ES = s.c.as<z64>();
  z64* M = s.d.as<z64>();
  frames_nn(pb, eta, F.Sinv.as<z64>(), 0, ES, 1.0, 0.0);
  frames_hn(pb, ES, ES, M);
  axpby<double>(st, pb->ntot * p, 1.0, ES, 0.0, out);
  frames_nn(pb, Phi_new, M, 0, out, -tau, 1.0);
}

// T_xi(v) = (v - R(xi) X) S^-1 with S X + X S = xi^H v + v^H xi, in the eigenbasis of S
void transport_general(eahp_problem* pb, const z64* Phi_new, const z64* xi, const z64* v, const RetractFactors& F,
                       z64* out) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  Scratch& s = pb->arena->s;
  s.c.ensure(sizeof(z64) * pb->ntot * p);
  s.d.ensure(sizeof(z64) * nk * pp);
  s.e.ensure(sizeof(z64) * nk * pp);
  z64* Wf = s.c.as<z64>();
  z64* Bm = s.d.as<z64>();
  z64* Tm = s.e.as<z64>();
  const z64* V = F.V.as<z64>();
  frames_hn(pb, xi, v, Bm);
  hermitize(st, p, Bm, p, pp, nk);  // (B + B^H) / 2
  // Tm = V^H Bh ; Bm = 2 Tm V  (= 2 V^H Bh V), all k at once
  gemm_hn<double>(st, p, p, p, V, p, Bm, p, Tm, p, 1.0, 0.0, pb->ws.gemm_part, nk, pp, pp, pp);
  gemm_nn<double>(st, p, p, p, Tm, p, V, p, 0, Bm, p, 2.0, 0.0, 0.0, nk, pp, pp, pp);
  lyap_divide(st, p, F.d.as<double>(), Bm, p, nk, p, pp);
  // X = V Xt V^H
  gemm_nn<double>(st, p, p, p, V, p, Bm, p, 0, Tm, p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  gemm_nn<double>(st, p, p, p, Tm, p, V, p, 1, Bm, p, 1.0, 0.0, 0.0, nk, pp, pp, pp);
  // W = v - Phi_new X ; out = W S^-1
  axpby<double>(st, pb->ntot * p, 1.0, v, 0.0, Wf);
  frames_nn(pb, Phi_new, Bm, 0, Wf, -1.0, 1.0);
  frames_nn(pb, Wf, F.Sinv.as<z64>(), 0, out, 1.0, 0.0);
}

// ---------------------------------------------------------------- EA gradient
void ea_gradient(eahp_problem* pb, const z64* Phi, const z64* X, z64* G) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  const int64_t pp = (int64_t)p * p;
  Scratch& s = pb->arena->s;
  s.d.ensure(sizeof(z64) * nk * pp);
  s.f.ensure(sizeof(z64) * nk * pp * 2);
  z64* M = s.d.as<z64>();
  frames_hn(pb, Phi, X, M);
  inverse(st, p, M, p, pp, s.f.as<z64>(), nk, pb->d_info.as<int>());
  axpby<double>(st, pb->ntot * p, 1.0, Phi, 0.0, G);
  frames_nn(pb, X, M, 0, G, -1.0, 1.0);
  HIPCK(hipMemcpyAsync(pb->h_info, pb->d_info.p, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (int ik = 0; ik < nk; ++ik)
    if (pb->h_info[ik]) fail(EAHP_EFOM, "Phi^H X is singular in the energy-adaptive gradient");
}

// ---------------------------------------------------------------- block FOM
// Templated on the precision T of everything of length n (Krylov basis V,
// W = H V, residual blocks, the H-applies, TPA and the Gram products); the
// q x q projected problem and its solution Y are kept in FP64 (A, Cj, Y).
namespace {

template <typename T>
FomWork<T>& fomwork(eahp_problem* pb) {
  if constexpr (sizeof(T) == 8) return pb->arena->fw64;
  else return pb->arena->fw32;
}

constexpr bool is_fp64(double) { return true; }
constexpr bool is_fp64(float) { return false; }

// C (a x b, ldc, FP64) = alpha A^H B over n rows of precision T
template <typename T>
void gram_into64(eahp_problem* pb, FomWork<T>& w, int64_t n, int a, int b, const cplx<T>* A, const cplx<T>* B, z64* C,
                 int64_t ldc) {
  hipStream_t st = pb->ctx->stream;
  if constexpr (sizeof(T) == 8) {
    gemm_hn<double>(st, n, a, b, A, n, B, n, C, ldc, 1.0, 0.0, pb->ws.gemm_part);
  } else {
    w.stage.ensure(sizeof(cplx<T>) * (size_t)a * b);
    gemm_hn<T>(st, n, a, b, A, n, B, n, w.stage.template as<cplx<T>>(), a, 1.0, 0.0, pb->ws.gemm_part);
    convert2d(st, a, b, w.stage.template as<cplx<T>>(), a, C, ldc);
  }
}

// Orthonormal basis of span(R) (n x c, ld n) by pivoted CholQR twice; written to
// dest (ld n).  Returns the rank.  The pivoted Cholesky runs in FP64 on the
// Gram matrix of precision T.
template <typename T>
int rrqr(eahp_problem* pb, int64_t n, int c, const cplx<T>* R, cplx<T>* dest, double tol, FomWork<T>& w) {
  hipStream_t st = pb->ctx->stream;
  if (c <= 0) return 0;
  w.Gm64.ensure(sizeof(z64) * c * c);
  w.PU64.ensure(sizeof(z64) * c * c);
  w.PU.ensure(sizeof(cplx<T>) * c * c);
  w.tmp.ensure(sizeof(cplx<T>) * n * c);
  w.piv.ensure(sizeof(int) * c);
  int* piv = w.piv.template as<int>();
  int* rank = pb->d_info.as<int>();
  cplx<T>* tmp = w.tmp.template as<cplx<T>>();
  auto factor = [&](const cplx<T>* X, int cols, double tl) {
    gram_into64<T>(pb, w, n, cols, cols, X, X, w.Gm64.template as<z64>(), cols);
    pchol_inv(st, cols, w.Gm64.template as<z64>(), cols, tl, piv, rank, w.PU64.template as<z64>(), cols, nullptr, pb->ws.chol);
    HIPCK(hipMemcpyAsync(pb->h_info, pb->d_info.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    const int r = pb->h_info[0];
    if constexpr (sizeof(T) == 4) convert2d(st, cols, std::max(r, 0), w.PU64.template as<z64>(), cols, w.PU.template as<c32>(), cols);
    return r;
  };
  auto pu = [&]() -> const cplx<T>* {
    if constexpr (sizeof(T) == 8) return w.PU64.template as<z64>();
    else return w.PU.template as<c32>();
  };
  const int r = factor(R, c, tol);
  if (r <= 0) return 0;
  gemm_nn<T>(st, n, c, r, R, n, pu(), c, 0, tmp, n, 1.0, 0.0, 0.0);
  // second pass
  const int r2 = factor(tmp, r, 0.0);
  gemm_nn<T>(st, n, r, r2, tmp, n, pu(), r, 0, dest, n, 1.0, 0.0, 0.0);
  return r2;
}

template <typename T>
void grow(hipStream_t st, FomWork<T>& w, int64_t n, int need, int p) {
  if (need <= w.qcap && n == w.n) return;
  const int old = (n == w.n) ? w.qcap : 0;
  const int cap = std::max(need, old + 4 * p);
  DevMem V2, W2, A2, C2;
  V2.alloc(sizeof(cplx<T>) * n * cap);
  W2.alloc(sizeof(cplx<T>) * n * cap);
  A2.alloc(sizeof(z64) * (size_t)cap * cap);
  C2.alloc(sizeof(z64) * (size_t)cap * p);
  if (old > 0) {
    HIPCK(hipMemcpyAsync(V2.p, w.V.p, sizeof(cplx<T>) * n * old, hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpyAsync(W2.p, w.W.p, sizeof(cplx<T>) * n * old, hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpy2DAsync(A2.p, sizeof(z64) * cap, w.A.p, sizeof(z64) * old, sizeof(z64) * old, old,
                           hipMemcpyDeviceToDevice, st));
    HIPCK(hipMemcpy2DAsync(C2.p, sizeof(z64) * cap, w.Cj.p, sizeof(z64) * old, sizeof(z64) * old, p,
                           hipMemcpyDeviceToDevice, st));
    HIPCK(hipStreamSynchronize(st));  // the old buffers are freed below
  }
  std::swap(w.V.p, V2.p);
  std::swap(w.V.bytes, V2.bytes);
  std::swap(w.W.p, W2.p);
  std::swap(w.W.bytes, W2.bytes);
  std::swap(w.A.p, A2.p);
  std::swap(w.A.bytes, A2.bytes);
  std::swap(w.Cj.p, C2.p);
  std::swap(w.Cj.bytes, C2.bytes);
  w.qcap = cap;
  w.n = n;
}

template <typename T>
double norm2(eahp_problem* pb, int64_t len, const cplx<T>* x) {
  dot_re(pb->ctx->stream, len, x, x, scal(pb, S_NRM), pb->ws.partial);
  fetch_scalars(pb, S_NRM + 1);
  return pb->h_scal[S_NRM];
}

// the context's second stream and events (created on first use, on its
// device; non-blocking, so that it overlaps a caller on the legacy default
// stream, with the order given by events only)
static const BandAux& band_aux(eahp_ctx* c) {
  static thread_local BandAux a;
  if (!c->aux_stream) {
    HIPCK(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
    for (auto& e : c->aux_ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  a.s = c->aux_stream;
  a.z = c->aux_ev[0];
  a.c = c->aux_ev[1];
  a.f = c->aux_ev[2];
  a.part = &c->aux_part;
  return a;
}

template <typename T>
FomInfo fom_k(eahp_problem* pb, int ik, const z64* Phi, const z64* R, const z64* Lam, double mu, double rtol,
              int maxit, double rank_tol, z64* X, const double* lw, const z64* lU) {
  hipStream_t st = pb->ctx->stream;
  FomWork<T>& w = fomwork<T>(pb);
  const int p = pb->p;
  auto& K = pb->kp[ik];
  const int64_t n = K.npw;
  const int64_t np_ = n * p;
  grow(st, w, n, 2 * p, p);
  w.C.ensure(sizeof(cplx<T>) * np_);
  w.E.ensure(sizeof(cplx<T>) * np_);
  w.Rj.ensure(sizeof(cplx<T>) * np_);
  w.Sig.ensure(sizeof(z64) * p * p);
  w.U.ensure(sizeof(z64) * p * p);
  w.s.ensure(sizeof(double) * p);
  w.alpha.ensure(sizeof(double) * p);
  cplx<T>* C = w.C.template as<cplx<T>>();
  cplx<T>* E = w.E.template as<cplx<T>>();
  cplx<T>* Rj = w.Rj.template as<cplx<T>>();
  auto Vp = [&]() { return w.V.template as<cplx<T>>(); };
  auto Wp = [&]() { return w.W.template as<cplx<T>>(); };
  // C = Phi - (H X0 - X0 Sigma) with X0 = Phi / mu equals -R / mu
  if constexpr (sizeof(T) == 8) {
    axpby<double>(st, np_, -1.0 / mu, R, 0.0, C);
  } else {
    convert<double>(st, np_, R, 1, C, 0);
    axpby<float>(st, np_, -1.0 / mu, C, 0.0, C);
  }
  const double nC2 = norm2<T>(pb, np_, C);
  // Sigma = Lambda - mu I and its eigendecomposition
  copy2d(st, p, p, Lam, p, w.Sig.template as<z64>(), p);
  add_diag(st, p, w.Sig.template as<z64>(), p, 0, -mu, 1);
  w.T1.ensure(sizeof(z64) * p * p);
  if (lw) {
    // Sigma = Lambda - mu I shares the eigenvectors of Lambda: s = w - mu
    affine(st, p, lw, -mu, 1.0, w.s.template as<double>());
    copy2d(st, p, p, lU, p, w.U.template as<z64>(), p);
  } else {
    copy2d(st, p, p, w.Sig.template as<z64>(), p, w.T1.template as<z64>(), p);
    heev(st, p, w.T1.template as<z64>(), p, 0, w.s.template as<double>(), 0, w.U.template as<z64>(), p, 0, 1, pb->d_info.as<int>(), pb->ws.eig);
  }
  // TPA: alpha_j = sum_G |k+G|^2/2 |phi_jG|^2
  col_weighted_norm2(st, n, p, Phi, n, K.d_kin.as<double>(), w.alpha.template as<double>());
  // V_1 = rrqr(P^-1 C), W_1 = H V_1
  tpa_apply<T>(st, n, p, K.d_kin.as<double>(), w.alpha.template as<double>(), C, n, Rj, n);
  int q = rrqr<T>(pb, n, p, Rj, Vp(), rank_tol, w);
  FomInfo info;
  if (q == 0) {
    axpby<double>(st, np_, 1.0 / mu, Phi, 0.0, X);
    info.relres = nC2 > 0 ? 1.0 : 0.0;
    return info;
  }
  apply_H_block<T>(pb, ik, q, Vp(), Wp());
  int ldA = w.qcap;
  gram_into64<T>(pb, w, n, q, q, Vp(), Wp(), w.A.template as<z64>(), ldA);
  gram_into64<T>(pb, w, n, q, p, Vp(), C, w.Cj.template as<z64>(), ldA);
  int it = 0;
  double relres = 1.0;
  const cplx<T>* Yt = nullptr;  // Y in precision T (q x p, ld q)
  for (;;) {
    ++it;
    ldA = w.qcap;
    // ---- projected Sylvester A_q Y - Y Sigma = C_q (FP64; in single precision
    // the reduction beyond q = 512 stores its trailing matrix in FP32)
    w.Ah.ensure(sizeof(z64) * q * q);
    w.T1.ensure(sizeof(cplx<T>) * q * p);
    w.T2.ensure(sizeof(z64) * q * p);
    w.Y.ensure(sizeof(z64) * q * p);
    w.YS.ensure(sizeof(z64) * q * p);
    // in the eigenbasis of Sigma: (A_q - s_l) y~_l = (C_q U)[:, l], then Y = Y~ U^H
    copy2d(st, q, q, w.A.template as<z64>(), ldA, w.Ah.template as<z64>(), q);
    gemm_nn<double>(st, q, p, p, w.Cj.template as<z64>(), ldA, w.U.template as<z64>(), p, 0, w.T2.template as<z64>(), q, 1.0, 0.0, 0.0);
    sylvester_tridiag(st, q, p, w.Ah.template as<z64>(), q, w.s.template as<double>(), w.T2.template as<z64>(), w.tri,
                      pb->ws.gemm_part, sizeof(T) == 4, &band_aux(pb->ctx));
    gemm_nn<double>(st, q, p, p, w.T2.template as<z64>(), q, w.U.template as<z64>(), p, 1, w.Y.template as<z64>(), q, 1.0, 0.0, 0.0);
    gemm_nn<double>(st, q, p, p, w.Y.template as<z64>(), q, w.Sig.template as<z64>(), p, 0, w.YS.template as<z64>(), q, 1.0, 0.0, 0.0);
    const cplx<T>* Ys;
    if constexpr (sizeof(T) == 8) {
      Yt = w.Y.template as<z64>();
      Ys = w.YS.template as<z64>();
    } else {
      w.YT.ensure(sizeof(c32) * q * p);
      w.YST.ensure(sizeof(c32) * q * p);
      convert<double>(st, (int64_t)q * p, w.Y.template as<z64>(), 1, w.YT.p, 0);
      convert<double>(st, (int64_t)q * p, w.YS.template as<z64>(), 1, w.YST.p, 0);
      Yt = w.YT.template as<c32>();
      Ys = w.YST.template as<c32>();
    }
    // ---- E = C - (W Y - V Y Sigma)
    axpby<T>(st, np_, 1.0, C, 0.0, E);
    gemm_nn<T>(st, n, q, p, Wp(), n, Yt, q, 0, E, n, -1.0, 0.0, 1.0);
    gemm_nn<T>(st, n, q, p, Vp(), n, Ys, q, 0, E, n, 1.0, 0.0, 1.0);
    const double nE2 = norm2<T>(pb, np_, E);
    relres = nC2 > 0 ? std::sqrt(nE2 / nC2) : 0.0;
    if (!std::isfinite(relres)) fail(EAHP_ENONFINITE, "non-finite residual in the metric solve");
    if (relres <= rtol || it >= maxit) break;
    // ---- R_j = (I - V V^H) P^-1 E_j, projected twice
    tpa_apply<T>(st, n, p, K.d_kin.as<double>(), w.alpha.template as<double>(), E, n, Rj, n);
    for (int pass = 0; pass < 2; ++pass) {
      gemm_hn<T>(st, n, q, p, Vp(), n, Rj, n, w.T1.template as<cplx<T>>(), q, 1.0, 0.0, pb->ws.gemm_part);
      gemm_nn<T>(st, n, q, p, Vp(), n, w.T1.template as<cplx<T>>(), q, 0, Rj, n, -1.0, 0.0, 1.0);
    }
    grow(st, w, n, q + p, p);
    ldA = w.qcap;
    cplx<T>* Vn = Vp() + (int64_t)q * n;
    const int r = rrqr<T>(pb, n, p, Rj, Vn, rank_tol, w);
    if (r == 0) break;
    cplx<T>* Wn = Wp() + (int64_t)q * n;
    apply_H_block<T>(pb, ik, r, Vn, Wn);
    // border A with V^H W_new (rows 0..q+r) and mirror; C_{j+1} = [C_j ; V_new^H C]
    gram_into64<T>(pb, w, n, q + r, r, Vp(), Wn, w.A.template as<z64>() + (int64_t)q * ldA, ldA);
    border_mirror(st, q, r, w.A.template as<z64>(), ldA);
    gram_into64<T>(pb, w, n, r, p, Vn, C, w.Cj.template as<z64>() + q, ldA);
    q += r;
    Yt = nullptr;
  }
  // X = X0 + V Y (Y is that of the last projected solve, of size q x p)
  axpby<double>(st, np_, 1.0 / mu, Phi, 0.0, X);
  if constexpr (sizeof(T) == 8) {
    gemm_nn<double>(st, n, q, p, Vp(), n, w.Y.template as<z64>(), q, 0, X, n, 1.0, 0.0, 1.0);
  } else {
    w.Xt.ensure(sizeof(c32) * np_);
    gemm_nn<float>(st, n, q, p, Vp(), n, w.YT.template as<c32>(), q, 0, w.Xt.template as<c32>(), n, 1.0, 0.0, 0.0);
    axpy_mixed(st, np_, 1.0, w.Xt.template as<c32>(), X);
  }
  info.iters = it;
  info.relres = relres;
  info.q = q;
  pb->fom_iters += it;
  return info;
}

}  // namespace

void metric_solve(eahp_problem* pb, const z64* Phi, const z64* R, const z64* Lam, double mu, double rtol, int maxit,
                  double rank_tol, z64* X, std::vector<FomInfo>* info, const LamEig* leig) {
  if (!(mu > 0)) fail(EAHP_EINVAL, "mu must be positive");
  if (info) info->clear();
  const int p = pb->p;
  const bool mixed = pb->precision == EAHP_MIXED;
  // the same deflation cut-off in both precisions: a direction whose pivot a
  // single-precision Gram matrix resolves poorly is still made orthonormal by
  // the second pass of CholQR2, and dropping fewer directions keeps the
  // single-precision Krylov spaces closer to the double-precision ones
  const double tol = rank_tol;
  if (pb->nk > 1 && p <= 128) {
    // every k-point at once (fom_batch.hip)
    LamEig own;
    if (!leig) {
      lambda_eig(pb, Lam, own);
      leig = &own;
    }
    std::vector<FomInfo> fi;
    if (mixed)
      fom_batch<float>(pb, Phi, R, leig->w.as<double>(), leig->U.as<z64>(), mu, rtol, maxit, tol, X, fi);
    else
      fom_batch<double>(pb, Phi, R, leig->w.as<double>(), leig->U.as<z64>(), mu, rtol, maxit, tol, X, fi);
    if (info) *info = fi;
    return;
  }
  for (int ik = 0; ik < pb->nk; ++ik) {
    const int64_t o = (int64_t)p * pb->kp[ik].off;
    const double* lw = leig ? leig->w.as<double>() + (int64_t)ik * p : nullptr;
    const z64* lU = leig ? leig->U.as<z64>() + (int64_t)ik * p * p : nullptr;
    const z64* L = Lam + (int64_t)ik * p * p;
    FomInfo fi = mixed ? fom_k<float>(pb, ik, Phi + o, R + o, L, mu, rtol, maxit, tol, X + o, lw, lU)
                       : fom_k<double>(pb, ik, Phi + o, R + o, L, mu, rtol, maxit, tol, X + o, lw, lU);
    if (info) info->push_back(fi);
  }
}

}  // namespace eahp
