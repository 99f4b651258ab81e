/*
 * eahp.h -- C ABI of the energy-adaptive Riemannian CG (EARCG) hot path for
 * plane-wave Kohn-Sham energy minimisation on the Stiefel manifold, on one
 * AMD MI355X (gfx950) GPU.
 *
 * The problem (Sec. 2.1, eq. (2.2), and its discrete product form, Sec. 5.1,
 * eq. (5.1)): minimise E(Psi) over Psi in St(p, n_1) x ... x St(p, n_K),
 * Psi_k^* Psi_k = I, with E the Kohn-Sham energy of eq. (1.1) in the Hartree
 * scaling of the experiments (H = -1/2 Laplacian + V_eff, doubly occupied
 * orbitals), a Gaussian local ionic potential, Hartree, Slater exchange and
 * one Gaussian s-projector per atom.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Orbital blocks ("frames"): device memory, complex values with interleaved
 *   real/imaginary parts (complex128 = 2 x double).  For k-point b the block
 *   is column-major n_b x p (orbital j contiguous, rows in the canonical
 *   plane-wave order: ascending linear FFT-box index (i1*n2 + i2)*n3 + i3 with
 *   i_d = m_d mod n_d); the blocks of successive k-points are concatenated, so
 *   block b starts at element p * offsets[b] (eahp_problem_layout).
 * p x p matrices (Lambda): device memory, nk consecutive column-major p x p
 *   complex128 matrices.
 * Ownership: the caller owns every buffer passed in; the library never frees
 *   caller memory.  Handles are library-owned and released by *_destroy.
 * Ordering: all device work is ordered on the context's HIP stream; every
 *   entry point that returns host scalars synchronises that stream before it
 *   returns.  Calls on one problem must not overlap (they share workspaces).
 * Errors: every int-returning function returns EAHP_OK (0) or a negative
 *   status; no exception crosses the ABI.  After an error the output buffers
 *   are unspecified and the handles stay valid.  eahp_strerror names a status;
 *   eahp_last_error returns a message for the calling thread's last error.
 */
#ifndef EAHP_H
#define EAHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EAHP_OK = 0,
  EAHP_EINVAL = -1,      /* bad argument (null pointer, size, layout)        */
  EAHP_ENOMEM = -2,      /* device or host allocation failed                 */
  EAHP_EDEVICE = -3,     /* HIP runtime error                                */
  EAHP_ENOTPD = -4,      /* Gram matrix of a retraction not positive definite*/
  EAHP_EFOM = -5,        /* metric solve broke down                          */
  EAHP_ELINESEARCH = -6, /* line search found no acceptable step             */
  EAHP_ENODESCENT = -7,  /* no descent direction after the reset rules       */
  EAHP_ENOCONV = -8,     /* solve reached maxit above tolerance              */
  EAHP_ENONFINITE = -9   /* NaN or Inf encountered                           */
};

enum { EAHP_FP64 = 0, EAHP_MIXED = 1 };
/* Outer iteration (eahp_solve_params.method) and retraction (.retraction). */
enum { EAHP_EARCG = 0, EAHP_EARGD = 1, EAHP_L2RCG = 2 };
enum { EAHP_POLAR = 0, EAHP_QR = 1 };

/* term switches of the Hamiltonian (all set = the full model) */
enum { EAHP_TERM_ION = 1, EAHP_TERM_HARTREE = 2, EAHP_TERM_XC = 4, EAHP_TERM_NONLOCAL = 8 };

typedef struct eahp_ctx eahp_ctx;
typedef struct eahp_problem eahp_problem;
typedef struct eahp_solver eahp_solver;

/* A crystal and its discretisation (Sec. 5.1).  All arrays are host memory
 * and are copied during eahp_problem_create. */
typedef struct {
  double lattice[9];     /* lattice vectors as columns: lattice[3*j+i] = (a_j)_i, bohr */
  int natoms;
  const double* frac;    /* natoms x 3 fractional positions (row-major)                */
  const double* Z;       /* natoms valence charges                                      */
  double r_loc;          /* Gaussian width of the local ionic potential (bohr)          */
  double r_proj;         /* width of the Gaussian s-projector (bohr)                    */
  double D_proj;         /* projector coupling D_I (Ha)                                 */
  double ecut;           /* kinetic cutoff |k+G|^2/2 <= ecut (Ha)                       */
  int fft[3];            /* FFT box; 0 = smallest 2/3/5-smooth n >= 4 max|m| + 1        */
  int nk;
  const double* kfrac;   /* nk x 3 fractional k-points (row-major)                      */
  const double* kweight; /* nk weights (sum 1)                                          */
  int p;                 /* orbitals per k-point                                        */
  double occ;            /* occupation per orbital (2 = doubly occupied)                */
  int precision;         /* EAHP_FP64 or EAHP_MIXED                                     */
  int terms;             /* bitwise or of EAHP_TERM_*                                   */
  /* Symmetry of a reduced k-point set (Sec. 5.1: the k-grid divided by the
   * symmetries of the crystal).  nsym <= 1: the k-set is used as given and the
   * density is not symmetrised.  nsym > 1: operations x -> W x + t on
   * fractional positions, as returned by eahp_symmetry_find; they must form a
   * group, map every atom onto an atom of the same charge (within 1e-4 bohr)
   * and map the FFT box onto itself (W_ab != 0 only where fft[a] = fft[b],
   * fft[a] t_a an integer), else EAHP_EINVAL.  The density of the k-set is
   * then averaged over the operations before the potentials are formed.    */
  int nsym;              /* number of operations, at most 4096                          */
  const int* sym_rot;    /* nsym x 9 integer rotations W, row-major (entries -1, 0, 1)  */
  const double* sym_trans; /* nsym x 3 fractional translations t                        */
} eahp_system_desc;

/* Method constants (Sec. 5.2: delta, sigma, gamma, eps, mu, FOM tolerance). */
typedef struct {
  double mu;         /* shift correction mu > 0 of Sigma = Lambda - mu I (Prop. 4.4)      */
  double fom_rtol;   /* relative residual at which the block FOM stops (2.5e-2)           */
  int fom_maxit;     /* block FOM iteration cap (per k-point)                             */
  double delta, sigma, gamma, eps; /* step-size parameters of Algorithm 2                 */
  int ls_maxit;      /* maximum energy evaluations per line search                        */
  double tol;        /* stop when ||R||_F <= tol                                          */
  int maxit;         /* outer iteration cap                                               */
  double mu_warm;    /* shift correction used while ||R||_F > warm_rtol (random starts)   */
  double warm_rtol;
  double rank_tol;   /* deflation threshold of the rank-revealing orthonormalisation      */
  int method;        /* EAHP_EARCG (Algorithm 3); EAHP_EARGD: the energy-adaptive          */
                     /* gradient -G as direction, an alternating Barzilai-Borwein step and */
                     /* non-monotone (Zhang-Hager) backtracking, the gradient-descent      */
                     /* method the paper compares against (Sec. 5.2); EAHP_L2RCG: CG on   */
                     /* the unpreconditioned L2 gradient R with the frozen-potential       */
                     /* Hessian step and the same backtracking (Sec. 5.2)                  */
  int retraction;    /* EAHP_POLAR (eq. (3.1)) or EAHP_QR (Gram-Schmidt, Sec. 3.1), with    */
                     /* the differentiated transport of the chosen retraction              */
  double nm_rho;     /* EARGD, L2RCG: accept tau when E(tau) <= C + nm_rho tau dE/dtau(0)  */
  double nm_backtrack; /* EARGD, L2RCG: tau <- nm_backtrack tau on rejection (0 < . < 1)   */
  double nm_theta;   /* EARGD, L2RCG: C_{k+1} = (theta Q_k C_k + E_{k+1}) / (theta Q_k + 1) */
} eahp_solve_params;

/* Statistics of eahp_solve (host memory, filled on return). */
typedef struct {
  int iters;            /* outer iterations done                         */
  int64_t napply;       /* orbital H-applies (one column at one k)       */
  int64_t napply_fp32;  /* of which in single precision                  */
  int ls_trials;        /* energy evaluations in all line searches       */
  int fom_iters;        /* block FOM iterations, summed over k and calls */
  double energy;        /* final energy                                  */
  double rnorm;         /* final ||R||_F                                 */
  double seconds;       /* wall time inside eahp_solve                   */
} eahp_stats;

/* Context: binds a device and a HIP stream (hipStream_t, may be NULL for the
 * null stream).  The stream is not owned. */
int eahp_ctx_create(int device, void* hip_stream, eahp_ctx** out);
void eahp_ctx_destroy(eahp_ctx* ctx);
int eahp_ctx_set_stream(eahp_ctx* ctx, void* hip_stream);

/* Builds the plane-wave bases (Sec. 5.1), the ionic potential on the FFT grid,
 * the projectors and all device workspaces. */
int eahp_problem_create(eahp_ctx* ctx, const eahp_system_desc* desc, eahp_problem** out);
void eahp_problem_destroy(eahp_problem* pb);

/* npw_per_k[nk], offsets[nk+1] (row offsets of the k-blocks), fft[3], p.
 * Any output pointer may be NULL. */
int eahp_problem_layout(const eahp_problem* pb, int64_t* npw_per_k, int64_t* offsets, int* fft, int* p);
int eahp_problem_nk(const eahp_problem* pb);
/* Device bytes held by the problem's workspaces. */
size_t eahp_problem_footprint(const eahp_problem* pb);

/* E(Psi) of eq. (1.1) (discrete form); terms (may be NULL) receives
 * [kinetic, nonlocal, ionic, Hartree, exchange].  Psi: frame, orthonormal. */
int eahp_energy(eahp_problem* pb, const void* Psi, double* E, double* terms);

/* Density rho(r) = sum_k w_k f sum_i |psi_ik(r)|^2 on the FFT grid (N_g reals,
 * layout (i1*n2+i2)*n3+i3), written to device buffer rho (may be NULL), and
 * V_eff = V_ion + V_H + V_x of that density, which becomes the problem's
 * current potential for eahp_apply_H. */
int eahp_density(eahp_problem* pb, const void* Psi, void* rho, void* Veff);

/* H_Psi X for a frame X (same layout as Psi): builds V_eff from the density of
 * Psi (Sec. 5.1), then applies kinetic + local (batched 3D FFTs) + nonlocal. */
int eahp_apply_H(eahp_problem* pb, const void* Psi, const void* X, void* HX);

/* Residual of the NLEVP (Sec. 2.2): Lambda_k = Hermitian part of
 * Psi_k^* (H Psi)_k (eq. (2.6)), R = H Psi - Psi Lambda; rnorm = ||R||_F,
 * E = energy.  R, Lambda, rnorm, E may each be NULL. */
int eahp_residual(eahp_problem* pb, const void* Psi, void* R, void* Lambda, double* rnorm, double* E);

/* Metric solve (Appendix A, Algorithm 4) per k-point: X solves
 * H_Psi X - X Sigma = Psi (eq. (5.2)) with Sigma = Lambda - mu I, X0 = Psi/mu,
 * TPA preconditioner, stopped at ||E_j||_F/||C||_F <= rtol or maxit.
 * iters_per_k, relres_per_k: host arrays of nk (may be NULL). */
int eahp_metric_solve(eahp_problem* pb, const void* Psi, double mu, double rtol, int maxit,
                      void* X, int* iters_per_k, double* relres_per_k);

/* Energy-adaptive gradient G = Psi - X (Psi^* X)^-1 per k (Sec. 5.2). */
int eahp_ea_gradient(eahp_problem* pb, const void* Psi, const void* X, void* G);

/* For callers that cannot allocate device memory (graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same G as
 * eahp_ea_gradient, with every intermediate (the p x p products and their
 * inverses, the partial tiles of the Gram product, the Gauss-Jordan work and
 * pivot flags) in a fixed device array of eahp_noalloc_scratch_bytes() bytes
 * (32 MiB) that the library holds on each device until the process ends; no
 * hipMalloc, hipFree or other allocation is made.  The array's address on a
 * device is looked up when the first context is created on that device.
 * Needs nk p^2 x 16 bytes (x 3 when p > 128) plus the Gram tiles to fit,
 * else EAHP_EINVAL before any device work.  All calls on one device share
 * the array: calls that overlap on one device (concurrent streams or host
 * threads) race and must be serialised by the caller.  Synchronises the
 * context stream (the singularity check, EAHP_EFOM). */
int eahp_ea_gradient_noalloc(eahp_problem* pb, const void* Psi, const void* X, void* G);
size_t eahp_noalloc_scratch_bytes(void);

/* Polar retraction Psi_out = pf(Psi + tau eta) (eqs. (3.1)-(3.2)), per k.
 * Returns EAHP_ENOTPD when (Psi + tau eta)^*(Psi + tau eta) is not positive
 * definite. */
int eahp_retract(eahp_problem* pb, const void* Psi, const void* eta, double tau, void* Psi_out);

/* Differentiated polar-retraction transport (Prop. 3.1, eqs. (3.3)-(3.4)):
 * Tv = T_xi(v) = (v - R(xi) X) S^-1 with S = sf(Psi + xi),
 * S X + X S = xi^* v + v^* xi. */
int eahp_transport(eahp_problem* pb, const void* Psi, const void* xi, const void* v, void* Tv);

/* qR retraction, the alternative the paper names in Sec. 3.1: Psi_out =
 * qf(Psi + tau eta), the Q factor of (Psi + tau eta) = Q R with R upper
 * triangular and positive on the diagonal, from the Cholesky factor of the
 * Gram matrix; EAHP_ENOTPD when a Gram matrix is not positive definite.
 * transport_qr: the differentiated qR retraction D qf(Psi + xi)[v]
 * (Tv tangent at qf(Psi + xi)).  Layouts and ownership as eahp_retract /
 * eahp_transport. */
int eahp_retract_qr(eahp_problem* pb, const void* Psi, const void* eta, double tau, void* Psi_out);
int eahp_transport_qr(eahp_problem* pb, const void* Psi, const void* xi, const void* v, void* Tv);

/* One line search (Algorithm 2) on f(t) = E(R_Psi(t eta)) from tau0;
 * on success tau, Psi_out = R_Psi(tau eta), trials (energy evaluations). */
int eahp_linesearch(eahp_problem* pb, const void* Psi, const void* eta, double tau0,
                    const eahp_solve_params* prm, double* tau, void* Psi_out, int* trials);

/* The control of Algorithm 2 alone, on the host, for a caller-supplied
 * f(t) (any smooth function of one variable with f'(0) < 0): fn(t, &f, &df,
 * user) returns 0 and writes f(t) and f'(t), or returns non-zero to abort
 * (EAHP_EINVAL).  f0 = f(0), df0 = f'(0).  The same readings as
 * eahp_linesearch (test, branches, bisection, ls_maxit); only prm->delta,
 * sigma, gamma, eps and ls_maxit are read.  On success tau is the accepted
 * step (the last point fn was called at) and trials the number of calls.
 * No device work. */
typedef int (*eahp_ls_eval)(double t, double* f, double* df, void* user);
int eahp_linesearch_host(double f0, double df0, double tau0, const eahp_solve_params* prm, eahp_ls_eval fn,
                         void* user, double* tau, int* trials);

/* Full EARCG solve (Algorithm 3) from Psi_inout (any full-rank frame: it is
 * orthonormalised by pf first); the minimiser is written back.  Returns
 * EAHP_ENOCONV (with Psi_inout holding the last iterate) at maxit. */
int eahp_solve(eahp_problem* pb, void* Psi_inout, const eahp_solve_params* prm, eahp_stats* stats);

/* Steppable form of eahp_solve (Algorithm 3): create evaluates the start
 * point pf(Psi0), its residual and its first energy-adaptive gradient; step
 * runs up to nsteps outer iterations (fewer when ||R||_F <= tol is reached)
 * and fills cumulative stats; it returns EAHP_ENOCONV while not converged.
 * The solver owns its frames (about 12 frames of device memory); Psi0 is not
 * retained.  get copies the current iterate (may be NULL) and its scalars. */
int eahp_solver_create(eahp_problem* pb, const void* Psi0, const eahp_solve_params* prm, eahp_solver** out);
int eahp_solver_step(eahp_solver* sv, int nsteps, eahp_stats* stats);
int eahp_solver_get(eahp_solver* sv, void* Psi_out, double* E, double* rnorm);
void eahp_solver_destroy(eahp_solver* sv);

/* Per-kernel timing with HIP events recorded on the context stream around
 * every launch of the H-apply kernels: 0 = inverse y/z plane transforms,
 * 1 = x-line transforms with the V_eff product, 2 = forward y/z transforms
 * with the gather and kinetic term, 3 = density x-line transforms; 4, 5, 6 =
 * the single-precision launches of 0, 1, 2 (metric solve of EAHP_MIXED);
 * 7 = the Householder reduction of the projected systems of the metric solve
 * beyond q = 512 (several work-groups, the trailing matrix in memory); and
 * around the complex matrix products (MFMA): 8 = A^H B in FP64,
 * 9 = A M in FP64, 10 = A^H B in FP32, 11 = A M in FP32, each over n >= 1024
 * rows (Gram matrices, projections, basis updates), 12..15 = the same over
 * fewer rows (products of the small projected matrices).
 * enable(1) starts recording (and resets); only one context records the
 * products at a time (the last one enabled).  read returns and resets the
 * summed duration, the launch count and, for 0..7, the algorithmic bytes
 * (compulsory loads and stores of each launch; for 7 one read and one write
 * of the live trailing matrix per step), for 8..15 the flops (8 per complex
 * multiply-add) since the last read. */
int eahp_prof_enable(eahp_ctx* ctx, int on);
int eahp_prof_read(eahp_ctx* ctx, int kernel, double* total_ms, int64_t* launches, double* bytes);

/* Frame H-applies as replayed HIP graphs (for callers that repeat the same
 * H-apply many times, such as the solver's line-search trials and the
 * serving loop, where the launch sequence and not the kernels costs the
 * time at small sizes).  With on = 1, the frame H-applies of this problem
 * (eahp_apply_H and those inside the solvers) are captured into a graph the
 * second time the same frames and workspaces occur and replayed from then
 * on; results are bit-for-bit those of the plain launches.  Requires a
 * context stream other than the legacy default stream (EAHP_EINVAL
 * otherwise).  on = 0 drops the captured graphs.  Kernel timing
 * (eahp_prof_enable) takes the plain launches.  graph_stats: graphs captured
 * and replays since the problem was created. */
int eahp_problem_set_graphs(eahp_problem* pb, int on);
int eahp_problem_graph_stats(const eahp_problem* pb, int64_t* captured, int64_t* replays);

/* Launch-configuration autotuner (process-wide).  Some kernels have several
 * valid launch configurations with identical results and a speed that depends
 * on the shape and the chip: the tile shape of the complex block products of
 * Secs. 5.1-5.2 and the work-group count of the multi-work-group Householder
 * reduction of large Hermitian matrices.  The table maps
 * "<arch>/<CUs> <kernel> <shape class>" to a choice.
 * enable(mode): 0 (the default) the default configuration everywhere (for
 * the block products: 64 x 16 or 64 x 32 tiles where the output has at most
 * 16 or 32 columns, which every mode keeps, else 64 x 64);
 * 1 the table's choice, and the first call in a class the table lacks times
 * every candidate on scratch outputs or copies of its inputs (extra device
 * allocations, the caller's stream synchronised) and keeps the fastest;
 * 2 the table's choices, nothing timed (classes it lacks take the default).
 * The first switch to mode 1 or 2 loads the file tune_table.txt beside the
 * library, if there is one.  EAHP_EINVAL for another mode.
 * load(path, added): adds the entries of a saved table (entries already
 * present are kept); *added (may be NULL) gets their number; EAHP_EINVAL if
 * the file cannot be read or a line is malformed.  save(path): writes the
 * table.  report writes the table as text, one line per class
 * ("<arch>/<CUs> <kernel> <class>: choice <c> ms <t0> <t1> ..."), into buf
 * (at most len bytes, NUL-terminated; buf may be NULL) and the size it
 * needs, NUL included, into *needed (may be NULL).  Host-only calls. */
int eahp_autotune_enable(int mode);
int eahp_autotune_load(const char* path, int* added);
int eahp_autotune_save(const char* path);
int eahp_autotune_report(char* buf, size_t len, size_t* needed);
/* Forces candidate `choice` (clamped to the last) of the tile shapes of the
 * complex block products for every later product, whether tuning is on or
 * not; -1 returns to the tuned or default choice.  The shapes give identical
 * results, so this only changes speed; it lets tests compare every shape.
 * Host-only call. */
int eahp_autotune_force(int choice);

/* Complex block products on device frames, the building blocks of Secs. 5.1
 * and 5.2 (Gram matrices V^* W, frame updates V Y), column-major:
 *   op 0: C (a x b, ldc) = A^H B + beta C, summed over n rows;
 *         A n x a (lda >= n), B n x b (ldb >= n);
 *   op 1: C (n x b, ldc) = A M + beta C; A n x a (lda >= n), M = B a x b
 *         (ldb >= a).
 * fp32 = 0: complex double, 1: complex float (interleaved re, im).  Products
 * of op 0 sum the row splits in a fixed order (same bits on every run); op 0
 * allocates its partial tiles for the call.  Runs on the context's stream
 * and returns after it has finished.  EAHP_EINVAL for a bad op, negative
 * size, short leading dimension or null operand. */
int eahp_block_product(eahp_ctx* ctx, int op, int fp32, int64_t n, int a, int b, const void* A, int64_t lda,
                       const void* B, int64_t ldb, void* C, int64_t ldc, double beta);

/* Layout of a system without touching the device: plane waves per k-point
 * (npw_per_k[nk], the row counts of the k-blocks of a frame), the FFT box and
 * an estimate of the device bytes one EARCG solve of it needs (frames, the
 * slab of a frame-wide H-apply, the block FOM, grids).  Any output may be
 * NULL.  Host-only; EAHP_EINVAL for an invalid description. */
int eahp_layout_estimate(const eahp_system_desc* desc, int64_t* npw_per_k, int fft[3], int64_t* bytes);

/* Serving loop over independent ground-state requests (Sec. 5 systems solved
 * to ||R||_F <= tol by Algorithm 3, each with its own system and frame).
 *
 * create: a scheduler for `device` that admits queued requests while their
 *   summed estimated footprints stay within hbm_budget bytes and fewer than
 *   max_slots run (a request larger than the budget runs alone).  Admitted
 *   requests run concurrently, each on its own stream from its own host
 *   thread, and keep all their state on the device until they finish.
 * submit: copies the description, the parameters and the initial frame
 *   (host memory, complex128, the layout of eahp_layout_estimate) and queues
 *   the request; *ticket identifies it.  Returns immediately.
 * poll: *state = 0 queued, 1 running, 2 done, 3 failed; once finished, the
 *   statistics, the latency from submission to completion and the time spent
 *   queued; returns the request's own status (EAHP_ENOCONV when maxit was
 *   reached) once finished, EAHP_OK before.
 * result: copies the final frame to host memory (same layout) and releases
 *   the ticket.  wait_all blocks until nothing is queued or running.
 * destroy waits for running requests, then frees everything.
 * A request's result is independent of the others in the mix: no reduction
 * crosses requests. */
typedef struct eahp_server eahp_server;
int eahp_server_create(int device, size_t hbm_budget, int max_slots, eahp_server** out);
int eahp_server_submit(eahp_server* srv, const eahp_system_desc* desc, const eahp_solve_params* prm,
                       const void* Psi0_host, uint64_t* ticket);
int eahp_server_poll(eahp_server* srv, uint64_t ticket, int* state, eahp_stats* stats, double* latency_s,
                     double* queued_s);
int eahp_server_result(eahp_server* srv, uint64_t ticket, void* Psi_host);
int eahp_server_wait_all(eahp_server* srv);
void eahp_server_destroy(eahp_server* srv);

/* ---------------------------------------------------------------- SCF comparator
 * Self-consistent field iteration, the method the paper compares EARCG with
 * and runs to make the experiments' initial guesses (Sec. 5.2): the p lowest
 * eigenpairs of every H_k at the potential of the current density (LOBPCG
 * with the TPA preconditioner), the output density, Anderson mixing of the
 * density (the nonlinear eigenvector problem of eq. (1.3) with the Aufbau
 * principle, Sec. 2.1).
 *
 * eahp_scf: Psi_inout (frame, device) is the start block on entry (any full-
 *   rank block per k) and the orthonormal eigenvector block of the last
 *   potential on return.  Returns EAHP_ENOCONV when maxit is reached above
 *   tol (Psi and stats are filled then too), EAHP_EINVAL for bad parameters
 *   or fewer than 3 p plane waves at a k-point.
 * eahp_eigensolve: the eigensolver alone: the potential is that of the
 *   density of Psi_pot (frame, device; NULL keeps the current potential of
 *   the problem); X_inout (frame) is the start block and receives the Ritz
 *   vectors; eigvals (host, nk x p, ascending per k), iters (host, summed
 *   over k) and rnorm (host, the largest ||H x - theta x||) may be NULL.    */
typedef struct {
  double tol;      /* stop when ||rho_out - rho_in||_2 over the cell <= tol               */
  int maxit;       /* SCF iterations                                                    */
  double beta;     /* damping of the mixed update, > 0                                   */
  int depth;       /* Anderson history length 1..16 (1: damped simple mixing)            */
  double eig_tol;  /* eigensolver stop: every ||H x - theta x|| <= eig_tol at every k;   */
                   /* 0: adaptive, 0.1 x the last density residual within [1e-12, 1e-2]; */
                   /* then tol counts only after a step solved to max(1e-12, 0.1 tol)   */
  int eig_maxit;   /* eigensolver iterations per k-point and SCF step                   */
} eahp_scf_params;
typedef struct {
  int iters;       /* SCF iterations done                                   */
  int64_t napply;  /* orbital H-applies (one column at one k)               */
  int eig_iters;   /* eigensolver iterations, summed over k and SCF steps   */
  double energy;   /* energy of the returned block                          */
  double res;      /* last ||rho_out - rho_in||_2                           */
  double seconds;  /* wall time inside eahp_scf                             */
} eahp_scf_stats;
int eahp_scf(eahp_problem* pb, void* Psi_inout, const eahp_scf_params* prm, eahp_scf_stats* stats);
int eahp_eigensolve(eahp_problem* pb, const void* Psi_pot, void* X_inout, double tol, int maxit, double* eigvals,
                    int* iters, double* rnorm);

/* ---------------------------------------------------------------- symmetry
 * Host-only helpers for symmetry-reduced k-point sets (Sec. 5.1: K is the
 * k1 k2 k3 points of the grid divided by the symmetries of the crystal).
 *
 * eahp_symmetry_find: the operations (W, t), x -> W x + t on fractional
 *   positions, that map the crystal of desc onto itself: W integer with
 *   entries in {-1, 0, 1} preserving the metric A^T A to 1e-8 relative, every
 *   atom mapped onto an atom of the same charge within symprec (bohr, modulo
 *   the lattice), and the FFT box of desc (fft[] = 0: the size eahp_problem_create
 *   would choose) mapped onto itself.  Pure translations of a non-primitive
 *   cell are operations too.  Order: W read row-major, lexicographic with
 *   -1 < 0 < 1, then t ascending; t in [0, 1) is a multiple of 1/fft[a].
 *   rot (max_ops x 9 ints) and trans (max_ops x 3 doubles) are host buffers
 *   of the caller; *nsym receives the count, and EAHP_EINVAL is returned when
 *   it exceeds max_ops (nothing is written to rot or trans then).
 * eahp_kpoints_reduce: the orbits of the nk fractional k-points under
 *   u -> W^T u for the distinct rotations of the nsym operations, and u -> -u
 *   when time_reversal != 0, points equal modulo integers (1e-8).  Keeps, in
 *   input order, the first point of every orbit with the summed weight of the
 *   orbit: kfrac_out (nk x 3) and kweight_out (nk) receive *nk_out points,
 *   kmap (nk) the kept index of every input point.  A set that is not closed
 *   under the operations is EAHP_EINVAL.  All buffers are host memory of the
 *   caller, sized for nk points.                                            */
int eahp_symmetry_find(const eahp_system_desc* desc, double symprec, int max_ops, int* rot, double* trans,
                       int* nsym);
int eahp_kpoints_reduce(int nsym, const int* rot, int time_reversal, int nk, const double* kfrac,
                        const double* kweight, double* kfrac_out, double* kweight_out, int* kmap, int* nk_out);

const char* eahp_strerror(int status);
const char* eahp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EAHP_H */
