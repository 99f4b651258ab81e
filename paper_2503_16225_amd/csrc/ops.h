// Host-side operators of the method (declarations shared by the .hip files).
#pragma once

#include <array>
#include <atomic>
#include <functional>
#include <string>

#include "kernels.h"

namespace eahp {

enum ScalarSlot {
  S_ION = 0, S_HART = 1, S_XC = 2, S_KIN = 3, S_NL = 4, S_RR = 5, S_DOT = 6, S_DOT2 = 7, S_DOT3 = 8,
  S_MIN = 9, S_NRM = 10, S_NRM2 = 11, kNumScal = 64
};

struct PointScalars {
  double E = 0, rnorm = 0;
  double terms[5] = {0, 0, 0, 0, 0};
};

extern thread_local std::string g_last_error;

// Timing of the complex products on the stream of the context whose timing is
// enabled (eahp_prof_enable; one context at a time): slot kProfGemm + op
// (0 A^H B, 1 A M) + 2 (FP32) + 4 (fewer than 1024 rows).
extern std::atomic<eahp_ctx*> g_prof_ctx;
// Autotuner (tune.hip): with tuning on, the first use of `key` runs every
// candidate 0..ncand-1 through run(c) (warm-up + timed, on scratch data) and
// keeps the fastest; with tuning off, candidate 0.
// While the stream is being captured into a graph, nothing is timed: the kept
// choice (or candidate 0) is returned.
bool autotune_on();
int autotune(hipStream_t st, const std::string& key, int ncand, const std::function<void(int)>& run);
// the kept choice of `key` with tuning on (candidate 0 otherwise), never timing
int autotune_kept(const std::string& key);
// the candidate forced by eahp_autotune_force (-1: none)
int autotune_forced();
// While one exists on a thread, autotune() on that thread times nothing (no
// allocation, no synchronisation): kept choices or candidate 0.
struct AutotuneHold {
  AutotuneHold();
  ~AutotuneHold();
  AutotuneHold(const AutotuneHold&) = delete;
  AutotuneHold& operator=(const AutotuneHold&) = delete;
};
// device address of this device's no-allocation scratch array (noalloc.hip)
void noalloc_init(int device);
void gemm_prof_begin(hipStream_t st, int slot);
void gemm_prof_end(hipStream_t st, int slot, double flops);

void build_problem(eahp_problem* pb, const eahp_system_desc* d);
void layout_estimate(const eahp_system_desc* d, std::vector<int64_t>& npw, int n[3], int& ns, size_t& bytes);
GridGeom geom(const eahp_problem* pb);
ColMap frame_map(const eahp_problem* pb);
ColMap block_map(const eahp_problem* pb, int k, int ncols);
void fetch_scalars(eahp_problem* pb, int n);
double* scal(eahp_problem* pb, int i);

// Crystal symmetry (symmetry.hip)
constexpr int kMaxSymOps = 4096;
struct SymOp {
  int W[9];     // row-major, fractional coordinates
  double t[3];  // fractional translation in [0, 1)
};
void find_symmetry(const eahp_system_desc* d, const int n[3], double symprec, std::vector<SymOp>& ops);
void reduce_kpoints(int nrot, const int* rot, bool time_reversal, int nk, const double* kfrac, const double* kw,
                    std::vector<double>& kout, std::vector<double>& wout, std::vector<int>& owner);
void setup_symmetry(eahp_problem* pb, const eahp_system_desc* d);  // validates, builds the box orbits
void symmetrize_density(eahp_problem* pb);                         // d_rho <- its orbit means

void potentials(eahp_problem* pb);
void density_potentials(eahp_problem* pb, const z64* Psi);
void apply_H_frame(eahp_problem* pb, const z64* X, z64* HX, bool tb_ready, double* nlvals);
template <typename T> void apply_H_block(eahp_problem* pb, int ik, int ncols, const cplx<T>* X, cplx<T>* HX);
// H X on a padded batch of k-point blocks (problem.hip): cpk columns of each
// of the nact k-points in kmap (device and host copies); block of k at
// k * kstride, columns with leading dimension ld.
template <typename T>
void apply_H_padded(eahp_problem* pb, int nact, const int* kmap_dev, const int* kmap_host, int cpk, const cplx<T>* X,
                    cplx<T>* HX, int64_t ld, int64_t kstride);
void evaluate_point(eahp_problem* pb, const z64* Psi, z64* HPsi, z64* R, z64* Lam, PointScalars* out);
void lambda_residual(eahp_problem* pb, const z64* Psi, const z64* HPsi, z64* R, z64* Lam);
// The per-k products of two frames (p columns, k-blocks stacked), every
// k-point in one launch: C_k = A_k^H B_k (p x p, C at stride p^2), and
// C_k = alpha A_k op(M_k) + beta C_k (M_k p x p at stride p^2; opM 1: M_k^H).
void frames_hn(eahp_problem* pb, const z64* A, const z64* B, z64* C);
void frames_nn(eahp_problem* pb, const z64* A, const z64* M, int opM, z64* C, double alpha, double beta);
double frame_dot(eahp_problem* pb, const z64* A, const z64* B);
double frame_dot_weighted(eahp_problem* pb, const z64* A, const z64* B);  // sum_k w_k Re tr(A_k^H B_k)
// Energy only (no H-apply); complete_point then adds H Psi, Lambda, R, ||R||_F.
void evaluate_energy(eahp_problem* pb, const z64* Psi, PointScalars* out);
void complete_point(eahp_problem* pb, const z64* Psi, z64* HPsi, z64* R, z64* Lam, PointScalars* out);

// Retraction factors per k: eigenvalues d of (Psi+xi)^H(Psi+xi), eigenvectors V, S^-1.
struct RetractFactors {
  DevMem d, V, Sinv;
};
void retract(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, z64* out, RetractFactors& F);
// qR retraction qf(Phi + tau eta) (R^-1 per k in F.Sinv) and its differentiated
// transport of v at the new point Q (uses F.Sinv of the same retraction).
void retract_qr(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, z64* out, RetractFactors& F);
void transport_qr(eahp_problem* pb, const z64* Q, const z64* v, const RetractFactors& F, z64* out);
// Retraction along a fixed direction eta at Phi: the Gram matrix of Phi + tau eta
// is S(tau) = (I + tau^2 eta^H eta) + Delta(tau) with the rounding-level
// Delta = (Phi^H Phi - I) + tau (Phi^H eta + eta^H Phi).  One eigendecomposition
// of eta^H eta = V diag(w) V^H serves every tau; S^-1/2 is taken to first
// order in Delta, which is exact to rounding while ||Delta|| stays tiny.
struct LineFactors {
  DevMem E0, A1, w, V, Dt, T;
};
void line_prepare(eahp_problem* pb, const z64* Phi, const z64* eta, LineFactors& L);
// pf(Phi + tau eta) from the line factors; false (nothing written) when Delta
// is too large for the first-order form, in which case retract() applies.
bool retract_line(eahp_problem* pb, const z64* Phi, const z64* eta, double tau, LineFactors& L, z64* out,
                  RetractFactors& F);
// Frame- and block-sized buffers of the manifold operations (per problem).
struct Scratch {
  DevMem a, b, c, d, e, f, g;
};
// Buffers of the block FOM at precision T (Krylov basis V, W = H V, the
// projected matrices, the rank-revealing step); they grow on demand.
template <typename T>
struct FomWork {
  DevMem V, W, A, Cj, C, E, Rj, Ah, T1, T2, Y, YS, YT, YST, Sig, U, s, alpha, Gm, Gm64, PU, PU64, tmp, piv, tri, stage,
      Xt;
  int64_t n = 0;
  int qcap = 0;
};
// Buffers of the block eigensolver of the SCF iteration (per problem).
struct LobWork {
  DevMem S, HS, T1, T2, T3, T4, R, A, V, w, C, Y, G, PU, piv, th, rn, alpha, idx;
  void ensure(int64_t n, int p);
};
// Buffers of the metric solve over all k-points at once (fom_batch.hip), at
// the precision of the Krylov blocks; k-blocks padded to a common ld.
struct FomBatchWork {
  DevMem C, E, Rj, Tmp, V, W, T1, stage;
  DevMem A, Cj, T2, Ct, Y, YS, YT, YST, wA, QA;
  DevMem Sig, s, alpha, Gm64, PU64, PU, piv, rank, kinp, kmap, live, done, norms, Xt, XP, eig, chol, tri;
  HostPinned hstage;  // host sources of the k-point lists uploaded without waiting
  int qcap = 0;
  int64_t ld = 0;
};
struct Arena {
  LobWork lob;
  Scratch s;
  LineFactors line;
  FomWork<double> fw64;
  FomWork<float> fw32;
  FomBatchWork fb64, fb32;
};

// Eigendecomposition of Lambda per k (w ascending order not guaranteed).
struct LamEig {
  DevMem w, U;
};
void lambda_eig(eahp_problem* pb, const z64* Lam, LamEig& E);
void transport_self(eahp_problem* pb, const z64* Phi_new, const z64* eta, double tau, const RetractFactors& F,
                    z64* out);
void transport_general(eahp_problem* pb, const z64* Phi_new, const z64* xi, const z64* v, const RetractFactors& F,
                       z64* out);
void ea_gradient(eahp_problem* pb, const z64* Phi, const z64* X, z64* G);
struct FomInfo {
  int iters = 0;
  double relres = 0;
  int q = 0;
};
// Algorithm 4 on every k-point; X out (frame); the potential must be that of Phi.
// SCF comparator (scf.hip): LOBPCG for the p lowest eigenpairs of H_k at the
// current potential (X: n_k x p block at k-point ik, in and out; theta: host,
// p Ritz values), and the SCF iteration with Anderson mixing on the frame Psi.
int lobpcg_k(eahp_problem* pb, int ik, z64* X, double tol, int maxit, double* theta, double* rnorm_max,
             int64_t* napply);
void scf_run(eahp_problem* pb, z64* Psi, const eahp_scf_params& prm, eahp_scf_stats* out);
void metric_solve(eahp_problem* pb, const z64* Phi, const z64* R, const z64* Lam, double mu, double rtol, int maxit,
                  double rank_tol, z64* X, std::vector<FomInfo>* info, const LamEig* leig = nullptr);
// Algorithm 4 on all k-points at once (fom_batch.hip); lw, lU: eigenvalues and
// eigenvectors of Lambda per k (nk x p, nk x p x p); info gets one entry per k.
template <typename T>
void fom_batch(eahp_problem* pb, const z64* Phi, const z64* R, const double* lw, const z64* lU, double mu, double rtol,
               int maxit, double rank_tol, z64* X, std::vector<FomInfo>& info);

}  // namespace eahp
