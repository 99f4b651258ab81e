// C entry points, the line search (Algorithm 2) and the EARCG driver
// (Algorithm 3).  Control flow runs on the host; every vector, matrix and
// reduction operation is a device kernel; only scalars (energies, pairings,
// norms, ranks) cross to the host.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ops.h"
#include "setup.h"

using namespace eahp;

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    f();
    return EAHP_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return EAHP_ENOMEM;
  } catch (...) {
    g_last_error = "unknown error";
    return EAHP_EDEVICE;
  }
}

z64* frame(eahp_problem* pb, int i) {
  pb->ws.f[i].ensure(sizeof(z64) * pb->ntot * pb->p);
  return pb->ws.f[i].as<z64>();
}

void check_problem(eahp_problem* pb) {
  if (!pb) fail(EAHP_EINVAL, "null problem");
  HIPCK(hipSetDevice(pb->ctx->device));
}

// ------------------------------------------------------------------ line search
struct Trial {
  z64 *Phi, *HPhi, *R, *Lam, *Teta;
  RetractFactors* F;
  PointScalars sc;
  double df;
};


// f(t), f'(t) at R_Phi(t eta) into the trial buffers (polar or qR retraction)
void eval_trial(eahp_problem* pb, const z64* Phi, const z64* eta, double t, Trial& tr, int retraction) {
  if (retraction == EAHP_QR) {
    retract_qr(pb, Phi, eta, t, tr.Phi, *tr.F);
  } else if (!retract_line(pb, Phi, eta, t, pb->arena->line, tr.Phi, *tr.F)) {
    retract(pb, Phi, eta, t, tr.Phi, *tr.F);
  }
  evaluate_point(pb, tr.Phi, tr.HPhi, tr.R, tr.Lam, &tr.sc);
  if (retraction == EAHP_QR) transport_qr(pb, tr.Phi, eta, *tr.F, tr.Teta);
  else transport_self(pb, tr.Phi, eta, t, *tr.F, tr.Teta);
  tr.df = frame_dot(pb, tr.R, tr.Teta);
  if (!std::isfinite(tr.df)) fail(EAHP_ENONFINITE, "non-finite slope in the line search");
}

// Modified secant step (Algorithm 2), in the printed order: the secant point
// of f' on [a, b] is evaluated, then (1) too high with f' < 0: tau = gamma b,
// [0, tau]; (2) left of a: tau = b / gamma, [0, tau]; (3) right of b: [b, tau];
// (4) inside: the half where f' changes sign.  Readings: approximate Wolfe
// test f <= f0 + eps|f0| and |f'| <= min(sigma, 1 - 2 delta)|f'(0)|; equal
// slopes take the midpoint; a kept bracket [a, tau] whose new right end has
// energy above the bound is bisected on the next trial.  ev(t, f, df)
// evaluates f and f' at t; the accepted point is always the last evaluated
// one.  Throws EAHP_ELINESEARCH after ls_maxit evaluations.
template <typename Eval>
double secant_core(Eval&& evf, double f0, double df0, double tau0, const eahp_solve_params& prm, int* trials_out) {
  const double c = std::min(prm.sigma, 1.0 - 2.0 * prm.delta);
  const double fbound = f0 + prm.eps * std::fabs(f0);
  int trials = 0;
  double ft = 0, dft = 0;
  auto ev = [&](double t) {
    if (trials >= prm.ls_maxit) fail(EAHP_ELINESEARCH, "line search: no acceptable step");
    ++trials;
    evf(t, ft, dft);
    if (!std::isfinite(ft) || !std::isfinite(dft)) fail(EAHP_ENONFINITE, "non-finite value in the line search");
  };
  auto ok = [&](double f, double df) { return f <= fbound && std::fabs(df) <= c * std::fabs(df0); };
  double a = 0.0, dfa = df0;
  double b = tau0;
  ev(b);
  double dfb = dft;
  double tau = b;
  bool bisect = false;
  while (!ok(ft, dft)) {
    const double den = dfb - dfa;
    if (bisect) tau = 0.5 * (a + b);
    else if (den != 0.0 && std::isfinite(den)) tau = (a * dfb - b * dfa) / den;
    else tau = 0.5 * (a + b);
    bisect = false;
    ev(tau);
    if (ft > fbound && dft < 0.0) {
      tau = prm.gamma * b;
      a = 0.0;
      dfa = df0;
      b = tau;
      ev(b);
      dfb = dft;
    } else if (tau < a) {
      tau = b / prm.gamma;
      a = 0.0;
      dfa = df0;
      b = tau;
      ev(b);
      dfb = dft;
    } else if (tau > b) {
      a = b;
      dfa = dfb;
      b = tau;
      dfb = dft;
    } else if (dft >= 0.0) {
      b = tau;
      dfb = dft;
      bisect = ft > fbound;
    } else {
      a = tau;
      dfa = dft;
    }
  }
  if (trials_out) *trials_out = trials;
  return tau;
}

double secant_step(eahp_problem* pb, const z64* Phi, const z64* eta, double f0, double df0, double tau0,
                   const eahp_solve_params& prm, Trial& tr, int* trials_out) {
  if (prm.retraction != EAHP_QR) line_prepare(pb, Phi, eta, pb->arena->line);
  return secant_core(
      [&](double t, double& f, double& df) {
        eval_trial(pb, Phi, eta, t, tr, prm.retraction);
        f = tr.sc.E;
        df = tr.df;
      },
      f0, df0, tau0, prm, trials_out);
}

}  // namespace

struct eahp_solver {
  eahp_problem* pb = nullptr;
  eahp_solve_params prm{};
  DevMem fr[12], lamA, lamB, lamw;
  LamEig le;
  RetractFactors Fa, Fb;
  RetractFactors* Ft = nullptr;
  z64 *Phi = nullptr, *HPhi = nullptr, *R = nullptr, *Phit = nullptr, *HPhit = nullptr, *Rt = nullptr;
  z64 *eta = nullptr, *G = nullptr, *X = nullptr, *Tetat = nullptr, *TG = nullptr, *xi = nullptr;
  z64 *Lam = nullptr, *Lamt = nullptr;
  PointScalars sc;
  double rn = 0, mu = 0, tau_prev = 1.0;
  double nmC = 0, nmQ = 1;  // EARGD, L2RCG: Zhang-Hager reference energy and its weight
  PointScalars sct;         // scalars of the last accepted trial
  int it = 0, ls_trials = 0, fom_iters = 0;
  int64_t napply = 0, napply32 = 0;
  double seconds = 0;
};

namespace {

bool solver_converged(const eahp_solver* sv) { return sv->rn <= sv->prm.tol; }

// Shift correction: the paper's mu once ||R||_F <= warm_rtol; before that
// max(mu_warm, lambda_max(Lambda) - min V_eff + 1), which makes every
// H - s_l (s_l eigenvalues of Sigma) positive definite because H >= min V_eff.
double mu_for(eahp_solver* sv, double r, const z64* Lam) {
  eahp_problem* pb = sv->pb;
  lambda_eig(pb, Lam, sv->le);  // also the eigenbasis of Sigma = Lambda - mu I for the FOM
  if (r <= sv->prm.warm_rtol) return sv->prm.mu;
  hipStream_t st = pb->ctx->stream;
  maxval(st, pb->nk * pb->p, sv->le.w.as<double>(), scal(pb, S_DOT2));
  minval_big(st, pb->Ng, pb->d_veff.as<double>(), scal(pb, S_DOT3), pb->ws.partial);
  fetch_scalars(pb, S_DOT3 + 1);
  return std::max(sv->prm.mu_warm, pb->h_scal[S_DOT2] - pb->h_scal[S_DOT3] + 1.0);
}

void solver_gradient(eahp_solver* sv, const z64* P, const z64* Rr, const z64* L, double m, z64* Gout) {
  eahp_problem* pb = sv->pb;
  metric_solve(pb, P, Rr, L, m, sv->prm.fom_rtol, sv->prm.fom_maxit, sv->prm.rank_tol, sv->X, nullptr, &sv->le);
  ea_gradient(pb, P, sv->X, Gout);
}

struct Counters {
  eahp_solver* sv;
  std::chrono::steady_clock::time_point t0;
  int64_t a0, a32;
  int f0;
  explicit Counters(eahp_solver* s)
      : sv(s), t0(std::chrono::steady_clock::now()), a0(s->pb->napply), a32(s->pb->napply32), f0(s->pb->fom_iters) {}
  ~Counters() {
    sv->napply += sv->pb->napply - a0;
    sv->napply32 += sv->pb->napply32 - a32;
    sv->fom_iters += sv->pb->fom_iters - f0;
    sv->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

void solver_init(eahp_solver* sv, const z64* Psi0) {
  eahp_problem* pb = sv->pb;
  Counters cnt(sv);
  const size_t fb = sizeof(z64) * pb->ntot * pb->p;
  for (auto& f : sv->fr) f.alloc(fb);
  const size_t lamb = sizeof(z64) * pb->nk * pb->p * pb->p;
  sv->lamA.alloc(lamb);
  sv->lamB.alloc(lamb);
  sv->Phi = sv->fr[0].as<z64>();
  sv->HPhi = sv->fr[1].as<z64>();
  sv->R = sv->fr[2].as<z64>();
  sv->Phit = sv->fr[3].as<z64>();
  sv->HPhit = sv->fr[4].as<z64>();
  sv->Rt = sv->fr[5].as<z64>();
  sv->eta = sv->fr[6].as<z64>();
  sv->G = sv->fr[7].as<z64>();
  sv->X = sv->fr[8].as<z64>();
  sv->Tetat = sv->fr[9].as<z64>();
  sv->TG = sv->fr[10].as<z64>();
  sv->xi = sv->fr[11].as<z64>();
  sv->Lam = sv->lamA.as<z64>();
  sv->Lamt = sv->lamB.as<z64>();
  sv->Ft = &sv->Fb;
  // Phi^(0) = pf(Psi0)
  retract(pb, Psi0, Psi0, 0.0, sv->Phi, sv->Fa);
  evaluate_point(pb, sv->Phi, sv->HPhi, sv->R, sv->Lam, &sv->sc);
  sv->rn = sv->sc.rnorm;
  if (sv->prm.method == EAHP_L2RCG) {
    axpby<double>(pb->ctx->stream, pb->ntot * pb->p, -1.0, sv->R, 0.0, sv->eta);
  } else {
    sv->mu = mu_for(sv, sv->rn, sv->Lam);
    solver_gradient(sv, sv->Phi, sv->R, sv->Lam, sv->mu, sv->G);
    axpby<double>(pb->ctx->stream, pb->ntot * pb->p, -1.0, sv->G, 0.0, sv->eta);
  }
  sv->tau_prev = 1.0;
  sv->nmC = sv->sc.E;
  sv->nmQ = 1.0;
}

double nonmonotone_step(eahp_solver* sv, double tau, double dE);

// One iteration of EARGD: d = -G, an alternating Barzilai-Borwein trial step
// from S = Phi_k - Phi_{k-1}, Y = G_k - G_{k-1} (the first iteration tries 1),
// clamped to [1e-10, 1e10], and backtracking until the energy passes the
// non-monotone test E <= C + rho tau dE/dtau(0) against the Zhang-Hager
// reference C.  Trials evaluate the energy only; the accepted point then gets
// H Phi and its residual.  Phit holds the previous iterate between iterations.
void solver_iterate_gd(eahp_solver* sv) {
  eahp_problem* pb = sv->pb;
  Counters cnt(sv);
  hipStream_t st = pb->ctx->stream;
  const int64_t N = pb->ntot * pb->p;
  const eahp_solve_params& prm = sv->prm;
  const double slope_scale = 2.0 * pb->occ;
  axpby<double>(st, N, -1.0, sv->G, 0.0, sv->eta);
  double dE = slope_scale * frame_dot_weighted(pb, sv->R, sv->eta);
  int doublings = 0;
  while (!(dE < 0.0)) {
    if (++doublings > 30) fail(EAHP_ENODESCENT, "no descent direction");
    sv->mu *= 2.0;
    evaluate_point(pb, sv->Phi, sv->HPhi, sv->R, sv->Lam, &sv->sc);  // makes V_eff current
    solver_gradient(sv, sv->Phi, sv->R, sv->Lam, sv->mu, sv->G);
    axpby<double>(st, N, -1.0, sv->G, 0.0, sv->eta);
    dE = slope_scale * frame_dot_weighted(pb, sv->R, sv->eta);
  }
  double tau = 1.0;
  if (sv->it > 0) {
    // S into xi, Y into Rt (both free here); TG holds G_{k-1}
    axpby<double>(st, N, 1.0, sv->Phi, 0.0, sv->xi);
    axpby<double>(st, N, -1.0, sv->Phit, 1.0, sv->xi);
    axpby<double>(st, N, 1.0, sv->G, 0.0, sv->Rt);
    axpby<double>(st, N, -1.0, sv->TG, 1.0, sv->Rt);
    const double sy = std::fabs(frame_dot(pb, sv->xi, sv->Rt));
    if (sy == 0.0) {
      tau = sv->tau_prev;
    } else {
      tau = (sv->it % 2 == 1) ? frame_dot(pb, sv->xi, sv->xi) / sy : sy / frame_dot(pb, sv->Rt, sv->Rt);
      tau = std::min(std::max(tau, 1e-10), 1e10);
    }
  }
  tau = nonmonotone_step(sv, tau, dE);
  std::swap(sv->Phi, sv->Phit);  // Phit keeps the previous iterate for the next step
  std::swap(sv->HPhi, sv->HPhit);
  std::swap(sv->R, sv->Rt);
  std::swap(sv->Lam, sv->Lamt);
  sv->sc = sv->sct;
  sv->rn = sv->sc.rnorm;
  sv->mu = mu_for(sv, sv->rn, sv->Lam);
  solver_gradient(sv, sv->Phi, sv->R, sv->Lam, sv->mu, sv->TG);
  std::swap(sv->G, sv->TG);  // TG keeps G_{k-1}
  sv->tau_prev = tau;
  ++sv->it;
}

// One outer iteration of Algorithm 3.
void solver_iterate(eahp_solver* sv) {
  eahp_problem* pb = sv->pb;
  Counters cnt(sv);
  hipStream_t st = pb->ctx->stream;
  const int64_t N = pb->ntot * pb->p;
  const eahp_solve_params& prm = sv->prm;
  double df0 = frame_dot(pb, sv->R, sv->eta);
  if (!(df0 < 0.0)) {
    // reset to the gradient direction; if that fails too, enlarge mu
    axpby<double>(st, N, -1.0, sv->G, 0.0, sv->eta);
    df0 = frame_dot(pb, sv->R, sv->eta);
    int doublings = 0;
    while (!(df0 < 0.0)) {
      if (++doublings > 30) fail(EAHP_ENODESCENT, "no descent direction");
      sv->mu *= 2.0;
      evaluate_point(pb, sv->Phi, sv->HPhi, sv->R, sv->Lam, &sv->sc);  // makes V_eff current
      solver_gradient(sv, sv->Phi, sv->R, sv->Lam, sv->mu, sv->G);
      axpby<double>(st, N, -1.0, sv->G, 0.0, sv->eta);
      df0 = frame_dot(pb, sv->R, sv->eta);
    }
  }
  Trial tr{sv->Phit, sv->HPhit, sv->Rt, sv->Lamt, sv->Tetat, sv->Ft, {}, 0};
  int trials = 0;
  const double tau = secant_step(pb, sv->Phi, sv->eta, sv->sc.E, df0, sv->tau_prev, prm, tr, &trials);
  sv->ls_trials += trials;
  const double rg = frame_dot(pb, sv->R, sv->G);
  // the accepted point is in the trial buffers (it was evaluated last)
  std::swap(sv->Phi, sv->Phit);
  std::swap(sv->HPhi, sv->HPhit);
  std::swap(sv->R, sv->Rt);
  std::swap(sv->Lam, sv->Lamt);
  RetractFactors* Facc = sv->Ft;
  sv->Ft = (sv->Ft == &sv->Fb) ? &sv->Fa : &sv->Fb;
  sv->sc = tr.sc;
  sv->rn = sv->sc.rnorm;
  sv->mu = mu_for(sv, sv->rn, sv->Lam);
  // T_{tau eta}(G_old), before eta and G change
  axpby<double>(st, N, tau, sv->eta, 0.0, sv->xi);
  if (prm.retraction == EAHP_QR) transport_qr(pb, sv->Phi, sv->G, *Facc, sv->TG);
  else transport_general(pb, sv->Phi, sv->xi, sv->G, *Facc, sv->TG);
  z64* Gn = sv->Phit;  // the previous point's buffer is free
  solver_gradient(sv, sv->Phi, sv->R, sv->Lam, sv->mu, Gn);
  const double rgn = frame_dot(pb, sv->R, Gn);
  const double rtg = frame_dot(pb, sv->R, sv->TG);
  const double fr = rgn / rg;
  const double prp = (rgn - rtg) / rg;
  const double beta = std::max(0.0, std::min(fr, prp));
  // eta = -G_new + beta T(eta)
  axpby<double>(st, N, -1.0, Gn, 0.0, sv->eta);
  axpby<double>(st, N, beta, sv->Tetat, 1.0, sv->eta);
  std::swap(sv->G, sv->Phit);
  sv->tau_prev = tau;
  ++sv->it;
}

// Energy-only trials of R_Phi(tau eta) with backtracking until the
// non-monotone test E <= C + rho tau dE passes; the accepted point is left
// in the trial buffers with H Phi, R, Lambda, and C, Q are updated.
double nonmonotone_step(eahp_solver* sv, double tau, double dE) {
  eahp_problem* pb = sv->pb;
  const eahp_solve_params& prm = sv->prm;
  int trials = 0;
  PointScalars sct;
  for (;;) {
    if (trials >= prm.ls_maxit) fail(EAHP_ELINESEARCH, "backtracking: no acceptable step");
    ++trials;
    if (prm.retraction == EAHP_QR) retract_qr(pb, sv->Phi, sv->eta, tau, sv->Phit, *sv->Ft);
    else retract(pb, sv->Phi, sv->eta, tau, sv->Phit, *sv->Ft);
    evaluate_energy(pb, sv->Phit, &sct);
    if (sct.E <= sv->nmC + prm.nm_rho * tau * dE) break;
    tau *= prm.nm_backtrack;
  }
  sv->ls_trials += trials;
  complete_point(pb, sv->Phit, sv->HPhit, sv->Rt, sv->Lamt, &sct);
  sv->sct = sct;
  const double Qn = prm.nm_theta * sv->nmQ + 1.0;
  sv->nmC = (prm.nm_theta * sv->nmQ * sv->nmC + sct.E) / Qn;
  sv->nmQ = Qn;
  return tau;
}

// One iteration of L2RCG: the L2 gradient R as the gradient (no metric solve,
// no preconditioner), the step from the quadratic model with the frozen-
// potential Hessian, tau = -dE / h with h = 2 f sum_k w_k Re tr(eta^H (H eta -
// eta Lambda)) (the previous step when h <= 0), safeguarded by non-monotone
// backtracking; eta+ = -R+ + beta T(eta) with the hybrid FR-PRP beta on R.
void solver_iterate_l2(eahp_solver* sv) {
  eahp_problem* pb = sv->pb;
  Counters cnt(sv);
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p;
  const int64_t N = pb->ntot * p;
  const eahp_solve_params& prm = sv->prm;
  if (!(frame_dot(pb, sv->R, sv->eta) < 0.0)) axpby<double>(st, N, -1.0, sv->R, 0.0, sv->eta);
  const double dE = 2.0 * pb->occ * frame_dot_weighted(pb, sv->R, sv->eta);
  // H eta - eta Lambda into G (unused by this method); V_eff is that of Phi
  z64* He = sv->G;
  apply_H_frame(pb, sv->eta, He, false, nullptr);
  frames_nn(pb, sv->eta, sv->Lam, 0, He, -1.0, 1.0);
  const double h = 2.0 * pb->occ * frame_dot_weighted(pb, sv->eta, He);
  double tau = h > 0.0 ? -dE / h : sv->tau_prev;
  tau = std::min(std::max(tau, 1e-10), 1e10);
  const double rr = frame_dot(pb, sv->R, sv->R);
  tau = nonmonotone_step(sv, tau, dE);
  // transports to the accepted point (trial buffers): T(eta) into Tetat, T(R) into TG
  RetractFactors* Facc = sv->Ft;
  axpby<double>(st, N, tau, sv->eta, 0.0, sv->xi);
  if (prm.retraction == EAHP_QR) {
    transport_qr(pb, sv->Phit, sv->eta, *Facc, sv->Tetat);
    transport_qr(pb, sv->Phit, sv->R, *Facc, sv->TG);
  } else {
    transport_self(pb, sv->Phit, sv->eta, tau, *Facc, sv->Tetat);
    transport_general(pb, sv->Phit, sv->xi, sv->R, *Facc, sv->TG);
  }
  std::swap(sv->Phi, sv->Phit);
  std::swap(sv->HPhi, sv->HPhit);
  std::swap(sv->R, sv->Rt);
  std::swap(sv->Lam, sv->Lamt);
  sv->sc = sv->sct;
  sv->rn = sv->sc.rnorm;
  const double rn2 = frame_dot(pb, sv->R, sv->R);
  const double rtr = frame_dot(pb, sv->R, sv->TG);
  const double beta = std::max(0.0, std::min(rn2 / rr, (rn2 - rtr) / rr));
  axpby<double>(st, N, -1.0, sv->R, 0.0, sv->eta);
  axpby<double>(st, N, beta, sv->Tetat, 1.0, sv->eta);
  sv->tau_prev = tau;
  ++sv->it;
}

void solver_stats(const eahp_solver* sv, eahp_stats* s) {
  s->iters = sv->it;
  s->napply = sv->napply;
  s->napply_fp32 = sv->napply32;
  s->ls_trials = sv->ls_trials;
  s->fom_iters = sv->fom_iters;
  s->energy = sv->sc.E;
  s->rnorm = sv->rn;
  s->seconds = sv->seconds;
}

}  // namespace

// ====================================================================== C API
extern "C" {

int eahp_scf(eahp_problem* pb, void* Psi_inout, const eahp_scf_params* prm, eahp_scf_stats* stats) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi_inout || !prm) fail(EAHP_EINVAL, "null argument");
    scf_run(pb, static_cast<z64*>(Psi_inout), *prm, stats);
  });
}

int eahp_eigensolve(eahp_problem* pb, const void* Psi_pot, void* X_inout, double tol, int maxit, double* eigvals,
                    int* iters, double* rnorm) {
  return guarded([&] {
    check_problem(pb);
    if (!X_inout || !(tol > 0) || maxit < 0) fail(EAHP_EINVAL, "bad argument");
    if (Psi_pot) density_potentials(pb, static_cast<const z64*>(Psi_pot));
    std::vector<double> th(pb->p);
    int64_t napply = 0;
    int its = 0;
    double rmax = 0;
    for (int ik = 0; ik < pb->nk; ++ik) {
      double r = 0;
      its += lobpcg_k(pb, ik, static_cast<z64*>(X_inout) + (int64_t)pb->p * pb->kp[ik].off, tol, maxit, th.data(),
                      &r, &napply);
      rmax = std::max(rmax, r);
      if (eigvals) std::memcpy(eigvals + (size_t)ik * pb->p, th.data(), sizeof(double) * pb->p);
    }
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
    if (iters) *iters = its;
    if (rnorm) *rnorm = rmax;
  });
}

int eahp_symmetry_find(const eahp_system_desc* desc, double symprec, int max_ops, int* rot, double* trans,
                       int* nsym) {
  return guarded([&] {
    if (!desc || !nsym || max_ops < 0 || (max_ops > 0 && (!rot || !trans))) fail(EAHP_EINVAL, "null argument");
    std::vector<int64_t> npw;
    int n[3], ns;
    size_t bytes;
    layout_estimate(desc, npw, n, ns, bytes);
    std::vector<SymOp> ops;
    find_symmetry(desc, n, symprec, ops);
    *nsym = (int)ops.size();
    if ((int)ops.size() > max_ops) fail(EAHP_EINVAL, "more operations than max_ops");
    for (size_t g = 0; g < ops.size(); ++g) {
      std::memcpy(rot + 9 * g, ops[g].W, sizeof(int) * 9);
      std::memcpy(trans + 3 * g, ops[g].t, sizeof(double) * 3);
    }
  });
}

int eahp_kpoints_reduce(int nsym, const int* rot, int time_reversal, int nk, const double* kfrac,
                        const double* kweight, double* kfrac_out, double* kweight_out, int* kmap, int* nk_out) {
  return guarded([&] {
    if (nsym < 0 || nk <= 0 || (nsym > 0 && !rot) || !kfrac || !kweight || !kfrac_out || !kweight_out || !kmap ||
        !nk_out)
      fail(EAHP_EINVAL, "null argument or empty set");
    const int ident[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::vector<double> kout, wout;
    std::vector<int> owner;
    reduce_kpoints(nsym > 0 ? nsym : 1, nsym > 0 ? rot : ident, time_reversal != 0, nk, kfrac, kweight, kout, wout,
                   owner);
    std::memcpy(kfrac_out, kout.data(), sizeof(double) * kout.size());
    std::memcpy(kweight_out, wout.data(), sizeof(double) * wout.size());
    std::memcpy(kmap, owner.data(), sizeof(int) * nk);
    *nk_out = (int)wout.size();
  });
}

const char* eahp_strerror(int s) {
  switch (s) {
    case EAHP_OK: return "ok";
    case EAHP_EINVAL: return "invalid argument";
    case EAHP_ENOMEM: return "out of memory";
    case EAHP_EDEVICE: return "HIP runtime error";
    case EAHP_ENOTPD: return "retraction Gram matrix not positive definite";
    case EAHP_EFOM: return "metric solve breakdown";
    case EAHP_ELINESEARCH: return "line search failed";
    case EAHP_ENODESCENT: return "no descent direction";
    case EAHP_ENOCONV: return "not converged";
    case EAHP_ENONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* eahp_last_error(void) { return g_last_error.c_str(); }

int eahp_ctx_create(int device, void* hip_stream, eahp_ctx** out) {
  return guarded([&] {
    if (!out) fail(EAHP_EINVAL, "null output");
    int n = 0;
    HIPCK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(EAHP_EINVAL, "no such device");
    HIPCK(hipSetDevice(device));
    noalloc_init(device);
    auto* c = new eahp_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
  });
}

void eahp_ctx_destroy(eahp_ctx* ctx) { delete ctx; }

int eahp_ctx_set_stream(eahp_ctx* ctx, void* hip_stream) {
  return guarded([&] {
    if (!ctx) fail(EAHP_EINVAL, "null context");
    ctx->stream = (hipStream_t)hip_stream;
  });
}

int eahp_problem_create(eahp_ctx* ctx, const eahp_system_desc* desc, eahp_problem** out) {
  eahp_problem* pb = nullptr;
  const int rc = guarded([&] {
    if (!ctx || !desc || !out) fail(EAHP_EINVAL, "null argument");
    HIPCK(hipSetDevice(ctx->device));
    pb = new eahp_problem;
    pb->ctx = ctx;
    pb->arena = new Arena;
    build_problem(pb, desc);
    *out = pb;
  });
  if (rc != EAHP_OK) delete pb;
  return rc;
}

void eahp_problem_destroy(eahp_problem* pb) {
  if (pb) {
    (void)hipSetDevice(pb->ctx->device);
    (void)hipStreamSynchronize(pb->ctx->stream);
  }
  delete pb;
}

int eahp_problem_nk(const eahp_problem* pb) { return pb ? pb->nk : 0; }

int eahp_problem_layout(const eahp_problem* pb, int64_t* npw, int64_t* offsets, int* fft, int* p) {
  return guarded([&] {
    if (!pb) fail(EAHP_EINVAL, "null problem");
    for (int k = 0; k < pb->nk; ++k) {
      if (npw) npw[k] = pb->kp[k].npw;
      if (offsets) offsets[k] = pb->kp[k].off;
    }
    if (offsets) offsets[pb->nk] = pb->ntot;
    if (fft)
      for (int d = 0; d < 3; ++d) fft[d] = pb->n[d];
    if (p) *p = pb->p;
  });
}

size_t eahp_problem_footprint(const eahp_problem* pb) {
  if (!pb) return 0;
  size_t b = pb->d_vion.bytes + pb->d_veff.bytes + pb->d_veff32.bytes + pb->d_rho.bytes + pb->d_box.bytes +
             pb->ws.planes.bytes + pb->ws.gemm_part.bytes + pb->ws.small.bytes + pb->ws.partial.bytes +
             pb->d_proj.bytes + pb->d_proj32.bytes;
  for (auto& K : pb->kp) b += K.d_kin.bytes + K.d_kin32.bytes + K.d_box.bytes;
  for (auto& f : pb->ws.f) b += f.bytes;
  return b;
}

int eahp_density(eahp_problem* pb, const void* Psi, void* rho, void* Veff) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi) fail(EAHP_EINVAL, "null frame");
    hipStream_t st = pb->ctx->stream;
    density_potentials(pb, (const z64*)Psi);
    if (rho) HIPCK(hipMemcpyAsync(rho, pb->d_rho.p, sizeof(double) * pb->Ng, hipMemcpyDeviceToDevice, st));
    if (Veff) HIPCK(hipMemcpyAsync(Veff, pb->d_veff.p, sizeof(double) * pb->Ng, hipMemcpyDeviceToDevice, st));
    HIPCK(hipStreamSynchronize(st));
  });
}

int eahp_energy(eahp_problem* pb, const void* Psi, double* E, double* terms) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !E) fail(EAHP_EINVAL, "null argument");
    PointScalars sc;
    DevMem lam;
    lam.alloc(sizeof(z64) * pb->nk * pb->p * pb->p);
    evaluate_point(pb, (const z64*)Psi, frame(pb, 0), frame(pb, 1), lam.as<z64>(), &sc);
    *E = sc.E;
    if (terms)
      for (int i = 0; i < 5; ++i) terms[i] = sc.terms[i];
  });
}

int eahp_apply_H(eahp_problem* pb, const void* Psi, const void* X, void* HX) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !X || !HX) fail(EAHP_EINVAL, "null argument");
    density_potentials(pb, (const z64*)Psi);
    apply_H_frame(pb, (const z64*)X, (z64*)HX, X == Psi, nullptr);
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_residual(eahp_problem* pb, const void* Psi, void* R, void* Lambda, double* rnorm, double* E) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi) fail(EAHP_EINVAL, "null frame");
    PointScalars sc;
    DevMem lam;
    z64* L = (z64*)Lambda;
    if (!L) {
      lam.alloc(sizeof(z64) * pb->nk * pb->p * pb->p);
      L = lam.as<z64>();
    }
    z64* Rb = R ? (z64*)R : frame(pb, 1);
    evaluate_point(pb, (const z64*)Psi, frame(pb, 0), Rb, L, &sc);
    if (rnorm) *rnorm = sc.rnorm;
    if (E) *E = sc.E;
  });
}

int eahp_metric_solve(eahp_problem* pb, const void* Psi, double mu, double rtol, int maxit, void* X, int* iters,
                      double* relres) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !X) fail(EAHP_EINVAL, "null argument");
    if (maxit <= 0 || !(rtol >= 0)) fail(EAHP_EINVAL, "bad FOM limits");
    DevMem lam;
    lam.alloc(sizeof(z64) * pb->nk * pb->p * pb->p);
    evaluate_point(pb, (const z64*)Psi, frame(pb, 0), frame(pb, 1), lam.as<z64>(), nullptr);
    std::vector<FomInfo> info;
    metric_solve(pb, (const z64*)Psi, frame(pb, 1), lam.as<z64>(), mu, rtol, maxit, 1e-7, (z64*)X, &info);
    for (int k = 0; k < pb->nk; ++k) {
      if (iters) iters[k] = info[k].iters;
      if (relres) relres[k] = info[k].relres;
    }
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_ea_gradient(eahp_problem* pb, const void* Psi, const void* X, void* G) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !X || !G) fail(EAHP_EINVAL, "null argument");
    ea_gradient(pb, (const z64*)Psi, (const z64*)X, (z64*)G);
  });
}

int eahp_retract(eahp_problem* pb, const void* Psi, const void* eta, double tau, void* Psi_out) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !eta || !Psi_out) fail(EAHP_EINVAL, "null argument");
    RetractFactors F;
    retract(pb, (const z64*)Psi, (const z64*)eta, tau, (z64*)Psi_out, F);
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_transport(eahp_problem* pb, const void* Psi, const void* xi, const void* v, void* Tv) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !xi || !v || !Tv) fail(EAHP_EINVAL, "null argument");
    RetractFactors F;
    z64* Pn = frame(pb, 2);
    retract(pb, (const z64*)Psi, (const z64*)xi, 1.0, Pn, F);
    transport_general(pb, Pn, (const z64*)xi, (const z64*)v, F, (z64*)Tv);
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_retract_qr(eahp_problem* pb, const void* Psi, const void* eta, double tau, void* Psi_out) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !eta || !Psi_out) fail(EAHP_EINVAL, "null argument");
    RetractFactors F;
    retract_qr(pb, (const z64*)Psi, (const z64*)eta, tau, (z64*)Psi_out, F);
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_transport_qr(eahp_problem* pb, const void* Psi, const void* xi, const void* v, void* Tv) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !xi || !v || !Tv) fail(EAHP_EINVAL, "null argument");
    RetractFactors F;
    z64* Pn = frame(pb, 2);
    retract_qr(pb, (const z64*)Psi, (const z64*)xi, 1.0, Pn, F);
    transport_qr(pb, Pn, (const z64*)v, F, (z64*)Tv);
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_linesearch(eahp_problem* pb, const void* Psi, const void* eta, double tau0, const eahp_solve_params* prm,
                    double* tau, void* Psi_out, int* trials) {
  return guarded([&] {
    check_problem(pb);
    if (!Psi || !eta || !prm || !tau) fail(EAHP_EINVAL, "null argument");
    DevMem lam0, lam1;
    lam0.alloc(sizeof(z64) * pb->nk * pb->p * pb->p);
    lam1.alloc(sizeof(z64) * pb->nk * pb->p * pb->p);
    PointScalars s0;
    evaluate_point(pb, (const z64*)Psi, frame(pb, 0), frame(pb, 1), lam0.as<z64>(), &s0);
    const double df0 = frame_dot(pb, frame(pb, 1), (const z64*)eta);
    if (!(df0 < 0)) fail(EAHP_ENODESCENT, "eta is not a descent direction");
    RetractFactors F;
    Trial tr{frame(pb, 2), frame(pb, 3), frame(pb, 4), lam1.as<z64>(), frame(pb, 5), &F, {}, 0};
    *tau = secant_step(pb, (const z64*)Psi, (const z64*)eta, s0.E, df0, tau0, *prm, tr, trials);
    if (Psi_out)
      HIPCK(hipMemcpyAsync(Psi_out, tr.Phi, sizeof(z64) * pb->ntot * pb->p, hipMemcpyDeviceToDevice, pb->ctx->stream));
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
  });
}

int eahp_linesearch_host(double f0, double df0, double tau0, const eahp_solve_params* prm, eahp_ls_eval fn,
                         void* user, double* tau, int* trials) {
  return guarded([&] {
    if (!prm || !fn || !tau) fail(EAHP_EINVAL, "null argument");
    if (!(df0 < 0)) fail(EAHP_ENODESCENT, "f'(0) is not negative");
    if (!(tau0 > 0) || !(prm->gamma > 0 && prm->gamma < 1) || prm->ls_maxit <= 0)
      fail(EAHP_EINVAL, "bad line-search parameters");
    *tau = secant_core(
        [&](double t, double& f, double& df) {
          if (fn(t, &f, &df, user) != 0) fail(EAHP_EINVAL, "evaluation callback failed");
        },
        f0, df0, tau0, *prm, trials);
  });
}

int eahp_solver_create(eahp_problem* pb, const void* Psi0, const eahp_solve_params* prmp, eahp_solver** out) {
  eahp_solver* sv = nullptr;
  const int rc = guarded([&] {
    check_problem(pb);
    if (!Psi0 || !prmp || !out) fail(EAHP_EINVAL, "null argument");
    const eahp_solve_params& prm = *prmp;
    if (!(prm.mu > 0) || !(prm.mu_warm > 0) || prm.fom_maxit <= 0 || prm.ls_maxit <= 0 ||
        !(prm.gamma > 0 && prm.gamma < 1))
      fail(EAHP_EINVAL, "bad solve parameters");
    if (prm.method != EAHP_EARCG && prm.method != EAHP_EARGD && prm.method != EAHP_L2RCG)
      fail(EAHP_EINVAL, "unknown method");
    if (prm.retraction != EAHP_POLAR && prm.retraction != EAHP_QR) fail(EAHP_EINVAL, "unknown retraction");
    if (prm.method != EAHP_EARCG &&
        !(prm.nm_rho > 0 && prm.nm_rho < 1 && prm.nm_backtrack > 0 && prm.nm_backtrack < 1 && prm.nm_theta >= 0 &&
          prm.nm_theta <= 1))
      fail(EAHP_EINVAL, "bad backtracking parameters");
    sv = new eahp_solver;
    sv->pb = pb;
    sv->prm = prm;
    solver_init(sv, (const z64*)Psi0);
    *out = sv;
  });
  if (rc != EAHP_OK) delete sv;
  return rc;
}

int eahp_solver_step(eahp_solver* sv, int nsteps, eahp_stats* stats) {
  int rc = guarded([&] {
    if (!sv) fail(EAHP_EINVAL, "null solver");
    check_problem(sv->pb);
    for (int i = 0; i < nsteps && !solver_converged(sv); ++i) {
      if (sv->prm.method == EAHP_EARGD) solver_iterate_gd(sv);
      else if (sv->prm.method == EAHP_L2RCG) solver_iterate_l2(sv);
      else solver_iterate(sv);
    }
  });
  if (sv && stats) solver_stats(sv, stats);
  if (rc == EAHP_OK && sv && !solver_converged(sv)) rc = EAHP_ENOCONV;
  return rc;
}

int eahp_solver_get(eahp_solver* sv, void* Psi_out, double* E, double* rnorm) {
  return guarded([&] {
    if (!sv) fail(EAHP_EINVAL, "null solver");
    if (Psi_out)
      HIPCK(hipMemcpyAsync(Psi_out, sv->Phi, sizeof(z64) * sv->pb->ntot * sv->pb->p, hipMemcpyDeviceToDevice,
                           sv->pb->ctx->stream));
    HIPCK(hipStreamSynchronize(sv->pb->ctx->stream));
    if (E) *E = sv->sc.E;
    if (rnorm) *rnorm = sv->rn;
  });
}

void eahp_solver_destroy(eahp_solver* sv) {
  if (sv) (void)hipStreamSynchronize(sv->pb->ctx->stream);
  delete sv;
}

int eahp_solve(eahp_problem* pb, void* Psi_inout, const eahp_solve_params* prmp, eahp_stats* stats) {
  eahp_solver* sv = nullptr;
  int rc = eahp_solver_create(pb, Psi_inout, prmp, &sv);
  if (rc != EAHP_OK) {
    if (stats) *stats = eahp_stats{};
    return rc;
  }
  rc = eahp_solver_step(sv, prmp->maxit, stats);
  const int rc2 = eahp_solver_get(sv, Psi_inout, nullptr, nullptr);
  eahp_solver_destroy(sv);
  return rc != EAHP_OK ? rc : rc2;
}

int eahp_problem_set_graphs(eahp_problem* pb, int on) {
  return guarded([&] {
    check_problem(pb);
    if (on && pb->ctx->stream == nullptr)
      fail(EAHP_EINVAL, "graph capture needs a stream other than the legacy default stream");
    HIPCK(hipStreamSynchronize(pb->ctx->stream));
    pb->graphs = on != 0;
    if (!on) pb->drop_graphs();
  });
}

int eahp_problem_graph_stats(const eahp_problem* pb, int64_t* captured, int64_t* replays) {
  return guarded([&] {
    if (!pb) fail(EAHP_EINVAL, "null problem");
    if (captured) *captured = pb->graph_captures;
    if (replays) *replays = pb->graph_replays;
  });
}

int eahp_block_product(eahp_ctx* ctx, int op, int fp32, int64_t n, int a, int b, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, double beta) {
  return guarded([&] {
    if (!ctx) fail(EAHP_EINVAL, "null context");
    if ((op != 0 && op != 1) || n < 0 || a < 0 || b < 0) fail(EAHP_EINVAL, "bad product operation or sizes");
    const int64_t rows_c = op == 0 ? a : n;
    if (lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, op == 0 ? n : a) ||
        ldc < std::max<int64_t>(1, rows_c))
      fail(EAHP_EINVAL, "leading dimension too small");
    const int64_t rows_b = op == 0 ? n : a;
    if ((n > 0 && a > 0 && !A) || (rows_b > 0 && b > 0 && !B) || (rows_c > 0 && b > 0 && !C))
      fail(EAHP_EINVAL, "null operand");
    HIPCK(hipSetDevice(ctx->device));
    DevMem part;
    hipStream_t st = ctx->stream;
    if (fp32) {
      if (op == 0)
        gemm_hn<float>(st, n, a, b, static_cast<const c32*>(A), lda, static_cast<const c32*>(B), ldb,
                       static_cast<c32*>(C), ldc, 1.0, beta, part);
      else
        gemm_nn<float>(st, n, a, b, static_cast<const c32*>(A), lda, static_cast<const c32*>(B), ldb, 0,
                       static_cast<c32*>(C), ldc, 1.0, 0.0, beta);
    } else {
      if (op == 0)
        gemm_hn<double>(st, n, a, b, static_cast<const z64*>(A), lda, static_cast<const z64*>(B), ldb,
                        static_cast<z64*>(C), ldc, 1.0, beta, part);
      else
        gemm_nn<double>(st, n, a, b, static_cast<const z64*>(A), lda, static_cast<const z64*>(B), ldb, 0,
                        static_cast<z64*>(C), ldc, 1.0, 0.0, beta);
    }
    HIPCK(hipStreamSynchronize(st));
  });
}

int eahp_prof_enable(eahp_ctx* ctx, int on) {
  return guarded([&] {
    if (!ctx) fail(EAHP_EINVAL, "null context");
    HIPCK(hipStreamSynchronize(ctx->stream));
    ctx->prof = on != 0;
    if (on) g_prof_ctx.store(ctx);
    else {
      eahp_ctx* expect = ctx;
      g_prof_ctx.compare_exchange_strong(expect, nullptr);
    }
    for (auto& s : ctx->slot) {
      s.used = 0;
      s.bytes = 0;
    }
  });
}

int eahp_prof_read(eahp_ctx* ctx, int kernel, double* total_ms, int64_t* launches, double* bytes) {
  return guarded([&] {
    if (!ctx || kernel < 0 || kernel >= kProfKernels) fail(EAHP_EINVAL, "bad kernel id");
    HIPCK(hipStreamSynchronize(ctx->stream));
    ProfSlot& s = ctx->slot[kernel];
    double tot = 0;
    for (int i = 0; i < s.used; ++i) {
      float ms = 0;
      HIPCK(hipEventElapsedTime(&ms, s.start[i], s.stop[i]));
      tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = s.used;
    if (bytes) *bytes = s.bytes;
    s.used = 0;
    s.bytes = 0;
  });
}

}  // extern "C"
