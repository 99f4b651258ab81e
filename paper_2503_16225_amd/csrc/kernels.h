// Launchers of the device kernels (host side).  All launches are asynchronous
// on the given stream; sizes are validated by the callers.
#pragma once

#include <mutex>

#include "internal.h"

namespace eahp {

// Per-k-point descriptor kept in device memory.
struct KDesc {
  int64_t npw;
  int64_t off;              // row offset of the k-block in a stacked frame
  const int* box;           // linear box index per plane wave
  const int* plane_start;   // ns + 1 row starts of the active planes
  const double* kin;        // |k+G|^2 / 2
  const float* kin32;
  const z64* proj;          // npw x natoms projectors (column-major)
  const c32* proj32;
  double w;                 // k-point weight
};

// Columns of an H-apply: column c is column j = c % cpk of the block of
// k-point k0 + c / cpk.  frame = 1: the block of k starts at cpk * off_k
// (a frame, ld npw_k); frame = 0: at 0 (one k-point's block, ld npw_k);
// frame = 2 (padded batch): the k-point is kmap[c / cpk], its block starts at
// k * kstride and every column has leading dimension ld (rows npw_k.. unused).
struct ColMap {
  const KDesc* kd;
  int k0;
  int cpk;
  int frame;
  int64_t ld = 0;
  int64_t kstride = 0;
  const int* kmap = nullptr;
};

struct GridGeom {
  int n1, n2, n3;
  int ns;              // active x-planes
  const int* plane_i1; // device: i1 of each active plane
  int ps;              // element stride between (y, z) planes of the slab buffer: n2 n3 rounded up to 16
  int m2max;           // largest |m2| of any plane wave: rows i2 = m2 mod n2 with |m2| > m2max stay zero
};

// ---- local-potential apply and density (hamiltonian.hip) -----------------
template <typename T>
void launch_inv_yz(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& pz,
                   const FftPlan& py, const cplx<T>* twz, const cplx<T>* twy, const cplx<T>* X, cplx<T>* Tb);
template <typename T>
void launch_x_local(hipStream_t st, int ncols, const GridGeom& g, const FftPlan& px, const cplx<T>* twx,
                    const T* V, cplx<T>* Tb);
template <typename T>
void launch_fwd_yz(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& pz,
                   const FftPlan& py, const cplx<T>* twz, const cplx<T>* twy, const cplx<T>* Tb, const cplx<T>* X,
                   cplx<T>* HX);
// rho(r) (+)= sum_c wgt(c) |psi_c(r)|^2, wgt(c) = w_k occ / Omega (FP64 only)
// (columns are split into groups that write partial densities to part, then summed in order)
void launch_x_density(hipStream_t st, const ColMap& cm, int ncols, const GridGeom& g, const FftPlan& px,
                      const z64* twx, const z64* Tb, double occ_over_omega, double* rho, int accumulate,
                      DevMem& part);

// ---- potentials on the full box (hamiltonian.hip) ---------------------------
void launch_box_fft(hipStream_t st, int n1, int n2, int n3, const FftPlan p[3], const z64* const tw[3],
                    z64* box, double sign);
void launch_rho_to_box(hipStream_t st, int64_t Ng, const double* rho, z64* box);
void launch_hartree_g(hipStream_t st, int n1, int n2, int n3, const double* B, z64* box);
// Veff = Vion + VH + Vx(rho); partial sums of Vion*rho, VH*rho/2, e_x(rho)
void launch_veff(hipStream_t st, int64_t Ng, const double* rho, const double* vion, const z64* vh_box,
                 int terms, double* veff, float* veff32, double* partial3, int nblocks);
void launch_real_part(hipStream_t st, int64_t Ng, const z64* box, double scale, double* out);

// ---- BLAS-like (blas.hip) ------------------------------------------------------
// C[a x b] = alpha * A^H B + beta * C over n rows; A lda, B ldb, C ldc (column-major).
template <typename T>
void gemm_hn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
             int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, DevMem& part, int batch = 1,
             int64_t sA = 0, int64_t sB = 0, int64_t sC = 0);
// The same product with a caller-given partial buffer of part_elems complex
// values (the row split is capped to fit; EAHP_EINVAL below
// gemm_hn_min_part(a, b, batch)), no allocation.
template <typename T>
void gemm_hn_mfma_ws(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* B,
                     int64_t ldb, cplx<T>* C, int64_t ldc, double alpha, double beta, cplx<T>* part, size_t part_elems,
                     int batch, int64_t sA, int64_t sB, int64_t sC);
size_t gemm_hn_min_part(int a, int b, int batch);
// tile order of gemm_hn / gemm_nn: 1 groups the tiles that share a block of
// the large operand on one die (its L2), 0 the plain order (same results)
void gemm_set_xcd_group(int on);
// C[n x b] = alpha * A[n x a] M[a x b] + beta * C ; opM: 0 = M, 1 = M^H
template <typename T>
void gemm_nn(hipStream_t st, int64_t n, int a, int b, const cplx<T>* A, int64_t lda, const cplx<T>* M, int64_t ldm,
             int opM, cplx<T>* C, int64_t ldc, double alpha_re, double alpha_im, double beta, int batch = 1,
             int64_t sA = 0, int64_t sM = 0, int64_t sC = 0);
// A ragged batch of per-k-point products: entry b is k-point k = kmap[b]
// (kmap null: k = b), whose n_k rows start at row off_k of stacked
// column-major operands (rows: (n_k, off_k) pairs in device memory).
// stacked = 0: the second operand of gemm_hn_ragged (the output of
// gemm_nn_ragged) is padded instead: block k at k times its stride, with the
// leading dimension given.
struct Ragged {
  const int64_t* rows = nullptr;
  const int* kmap = nullptr;
  int stacked = 1;
};
// C_b (a x b, ldc, at b sC) = alpha A_k^H B_k + beta C_b, A_k (n_k x a) at
// A + a off_k with leading dimension n_k, B_k stacked (at B + b off_k, leading
// dimension n_k) or padded (at B + k sB, ldb); nmax >= every n_k, ntot = the
// rows of all entries (for the rate).
template <typename T>
void gemm_hn_ragged(hipStream_t st, const Ragged& rg, int64_t nmax, int64_t ntot, int a, int b, const cplx<T>* A,
                    const cplx<T>* B, int64_t ldb, int64_t sB, cplx<T>* C, int64_t ldc, int64_t sC, double alpha,
                    double beta, DevMem& part, int batch);
// C_k = alpha A_k op(M_b) + beta C_k (opM 1: M_b^H), M_b at M + b sM, C_k
// stacked (at C + b off_k, leading dimension n_k) or padded (at C + k sC, ldc)
template <typename T>
void gemm_nn_ragged(hipStream_t st, const Ragged& rg, int64_t nmax, int64_t ntot, int a, int b, const cplx<T>* A,
                    const cplx<T>* M, int64_t ldm, int64_t sM, int opM, cplx<T>* C, int64_t ldc, int64_t sC,
                    double alpha, double beta, int batch);
// y = a x + b y (complex, length n, real coefficients)
template <typename T>
void axpby(hipStream_t st, int64_t n, double a, const cplx<T>* x, double b, cplx<T>* y);
// out = Re sum conj(x) y over n, deterministic (partials in part)
void dot_re(hipStream_t st, int64_t n, const z64* x, const z64* y, double* out_dev, DevMem& part);
void dot_re(hipStream_t st, int64_t n, const c32* x, const c32* y, double* out_dev, DevMem& part);  // FP64 sums
// 2-D copies between precisions (column-major, leading dimensions lds / ldd)
void convert2d(hipStream_t st, int rows, int cols, const c32* src, int64_t lds, z64* dst, int64_t ldd);
void convert2d(hipStream_t st, int rows, int cols, const z64* src, int64_t lds, c32* dst, int64_t ldd);
// y += a x, x single and y double precision
void axpy_mixed(hipStream_t st, int64_t n, double a, const c32* x, z64* y);
// out[k p + j] = sum_g w[g] |X_k[g, j]|^2 over the k-blocks of a stacked frame
// (w: the kinetic energies of k-point k when kin, else 1), one launch
void frame_col_wnorm2(hipStream_t st, const KDesc* kd, int nk, int p, const z64* X, int kin, double* out);
// out[j] = sum_g w[g] |x[g, j]|^2 (column reductions), or with w == null plain norms
void col_weighted_norm2(hipStream_t st, int64_t n, int ncols, const z64* X, int64_t ldx, const double* w,
                        double* out);
template <typename T>
void convert(hipStream_t st, int64_t n, const void* src, int src_fp64, void* dst, int dst_fp64);
// TPA preconditioner: Y[:, j] = X[:, j] / (kin + alpha_j)
template <typename T>
void tpa_apply(hipStream_t st, int64_t n, int ncols, const double* kin, const double* alpha, const cplx<T>* X,
               int64_t ldx, cplx<T>* Y, int64_t ldy);
// D-scaling of projector coefficients: B[I, j] *= D[I]
template <typename T>
void scale_rows(hipStream_t st, int m, int ncols, const double* D, cplx<T>* B, int64_t ldb);

// ---- small dense (dense.hip) ---------------------------------------------------
// Hermitian eigendecomposition A = V diag(w) V^H, w ascending (batch of
// matrices at strides sA, sw, sV): n <= 128 one work-group per matrix
// (Householder + divide and conquer in LDS); n <= 2048 Householder on
// several work-groups + divide and conquer in global memory (one matrix at a
// time, synchronises the stream); larger n cyclic Jacobi (A overwritten,
// EAHP_ENOCONV after 40 sweeps).  info: device int per matrix (Jacobi only).
void heev(hipStream_t st, int n, z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V, int64_t ldv,
          int64_t sV, int batch, int* info, DevMem& scr);
// In-place inverse of a general n x n matrix (Gauss-Jordan, partial pivoting):
// n <= 128 one work-group per matrix with the matrix in registers; larger n
// one matrix at a time on a cooperative grid (work: n x 2n per matrix;
// synchronises the stream).  info: device int per matrix, 1 when a pivot is 0.
void inverse(hipStream_t st, int n, z64* A, int64_t lda, int64_t sA, z64* work, int batch, int* info);
// Pivoted Cholesky of a Hermitian PSD G (n x n): G[piv, piv] = L L^H with rank r
// (diagonal pivots below tol * first pivot are dropped); outputs the upper
// triangular inverse factor U = L^-H padded (n x r), piv and r.  With pivot =
// false the pivots are taken in order (piv = identity, G = L L^H, U = R^-1 for
// the Cholesky factor R = L^H) and r is the number of positive pivots before
// the first non-positive one.
void pchol_inv(hipStream_t st, int n, z64* G, int64_t ldg, double tol, int* piv, int* rank, z64* Uinv,
               int64_t ldu, int* info, DevMem& scr, bool pivot = true);
// A batch of pivoted factorisations as above (n <= 128): matrix b at G + b sG,
// piv + b n, rank + b, U + b sU (n x n, columns beyond the rank zeroed).
void pchol_inv_batched(hipStream_t st, int n, const z64* G, int64_t ldg, int64_t sG, double tol, int* piv, int* rank,
                       z64* U, int64_t ldu, int64_t sU, int batch, DevMem& scr);
// qR retraction support: D = Omega(M) - M for a p x p M (batch), where Omega is the
// skew-Hermitian matrix with the strictly lower triangle of M, minus its
// conjugate transpose above, and i Im(M_jj) on the diagonal.
void qr_omega_minus(hipStream_t st, int p, const z64* M, int64_t ldm, int64_t sM, z64* D, int64_t ldd, int64_t sD,
                    int batch);
// Elementwise helpers on small matrices (n x m, column-major).
// Y = Q^H C U-ish products use gemm; these handle the spectral divisions.
void sylv_divide(hipStream_t st, int q, int p, const double* w, const double* s, z64* Y, int64_t ldy);
void lyap_divide(hipStream_t st, int p, const double* d, z64* X, int64_t ldx, int batch, int64_t sd, int64_t sX);
// M = V f(d) V^H with f(d) = d^e (e in {0.5, -0.5, -1}); batch over k
void spectral_fn(hipStream_t st, int p, const z64* V, int64_t ldv, int64_t sV, const double* d, int64_t sd,
                 double e, z64* M, int64_t ldm, int64_t sM, int batch);
// First-order inverse square root in a fixed eigenbasis (p x p blocks, ld p,
// batch over k): d = 1 + tau^2 w, Mt = diag(d^-1/2) - Dt o K (see dense.hip).
void polar_first_order(hipStream_t st, int p, const double* w, double tau, const z64* Dt, double* d, z64* Mt,
                       int batch);
void hermitize(hipStream_t st, int p, z64* M, int64_t ldm, int64_t sM, int batch);
// y = a + b x elementwise (n doubles)
void affine(hipStream_t st, int n, const double* x, double a, double b, double* y);
void add_diag(hipStream_t st, int p, z64* M, int64_t ldm, int64_t sM, double v, int batch);
void set_identity(hipStream_t st, int p, z64* M, int64_t ldm);
// (A - s_l I) y_l = c_l for all columns of Yt (q x p, ld q; overwritten by the
// solutions) through one Householder tridiagonalisation of A (destroyed).
// store32: for q > 512, the reduction keeps the trailing matrix in single
// precision (the single-precision metric solve).
// A second stream (default priority) and two events for work that overlaps the
// main stream's (the band reduction's look-ahead); owned by a context.
struct BandAux {
  hipStream_t s = nullptr;
  hipEvent_t z = nullptr, c = nullptr, f = nullptr;
  DevMem* part = nullptr;  // split-K partials of the products on s
};
void sylvester_tridiag(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws,
                       DevMem& part, bool store32 = false, const BandAux* aux = nullptr);
// Householder reduction of a Hermitian A (q x q, ld lda; destroyed for q > 512)
// to the Hermitian tridiagonal T = Q^H A Q, Q = H_0 ... H_{q-2}: dd (q reals,
// the diagonal), e (q complex, e[k] = T[k+1][k]), the reflectors Vh (q x q,
// ld q, v_k in rows k+1.. of column k) and beta (q); H_k = I - beta_k v_k v_k^H.
// scr: tridiag_scratch(q) bytes of device memory.  Synchronises the stream.
size_t tridiag_scratch(int q);
// held around every launch of a kernel whose work-groups wait on each other
std::mutex& coop_mutex();
void tridiag_reduce(hipStream_t st, int q, z64* A, int64_t lda, double* dd, z64* e, z64* Vh, double* beta, void* scr);
// The same for q > 512 with A held in single precision (destroyed); every
// step computes in FP64 and rounds the updated trailing entries to FP32.
void tridiag_reduce(hipStream_t st, int q, c32* A, int64_t lda, double* dd, z64* e, z64* Vh, double* beta, void* scr);
// The solve of sylvester_tridiag for nb matrices of order 2 <= q <= 512 at
// once: A_b (q x q, ld lda, stride sA; kept), Y_b (q x p, ld q, stride q p;
// overwritten by the solutions of (A_b - s[b p + l] I) y_l = y_l).  The
// reductions run as few cooperative launches as the resident work-groups
// allow.  ws grows to sylvester_tridiag_batched_scratch(q, p, nb) bytes.
// Synchronises the stream.
size_t sylvester_tridiag_batched_scratch(int q, int p, int nb);
void sylvester_tridiag_batched(hipStream_t st, int q, int p, int nb, const z64* A, int64_t lda, int64_t sA,
                               const double* s, z64* Y, DevMem& ws);
// Y <- Q^H Y (forward = 1) or Q Y (forward = 0) for the reflectors of tridiag_reduce;
// for q > 512 with wy_scr and part given: blocked products (MFMA), where
// wy_scr holds (ceil((q-1)/256) 256^2 + 256 ncols) complex values + 512 bytes
void apply_refl(hipStream_t st, int q, int ncols, const z64* Vh, const double* beta, z64* Y, int64_t ldy, int forward,
                void* wy_scr = nullptr, DevMem* part = nullptr);
// Y <- Q^H Y (forward = 1) or Q Y for Q = H_0 ... H_{q-off-1}, reflector k
// (column k of Vh, ld q, zero above row k + off) acting on rows k + off ..;
// scr: refl_blocked_scratch(q - off, ncols) bytes.
size_t refl_blocked_scratch(int nref, int ncols);
// apply_refl's register kernel over nb matrices: Vh_b at stride q^2 (ld q),
// beta_b at q, Y_b at sY; q <= 1536
void apply_refl_batched(hipStream_t st, int q, int ncols, int nb, const z64* Vh, const double* beta, z64* Y,
                        int64_t ldy, int64_t sY, int forward);
// apply_refl_blocked in two parts: the Gram matrices and triangular factors
// of the blocks into scr, then the products on ncols columns of Y with zs
// (2 x 256 x ncols values) for the intermediate blocks; the second part may
// run on several streams at once on disjoint columns, each with its own zs
// and part
void refl_blocked_prepare(hipStream_t st, int q, int off, const z64* Vh, const double* beta, void* scr, DevMem& part);
void refl_blocked_apply(hipStream_t st, int q, int off, int ncols, const z64* Vh, z64* Y, int64_t ldy, int forward,
                        const void* scr, z64* zs, DevMem& part);
void apply_refl_blocked(hipStream_t st, int q, int off, int ncols, const z64* Vh, const double* beta, z64* Y,
                        int64_t ldy, int forward, void* scr, DevMem& part);
// (A - s_l I) y_l = c_l for all columns of Yt (q x p, ld q; overwritten by the
// solutions) through a reduction of A (destroyed) to Hermitian band form and
// banded solves with partial pivoting (band.hip); q > 64.
// With aux: the trailing update of each panel beyond the next panel's
// columns runs on aux.s while the next panel is factored (identical results).
void sylvester_band(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws,
                    DevMem& part, const BandAux* aux = nullptr);

}  // namespace eahp
