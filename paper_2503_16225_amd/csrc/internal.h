// Internal declarations of the EARCG hot-path library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/eahp.h"

namespace eahp {

// ---------------------------------------------------------------- errors
struct Error {
  int status;
  std::string msg;
};
[[noreturn]] void fail(int status, const std::string& msg);
void hip_check(hipError_t e, const char* what, int line);
#define HIPCK(x) ::eahp::hip_check((x), #x, __LINE__)

// ---------------------------------------------------------------- complex
template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <typename T> using cplx = typename C2<T>::type;
using z64 = double2;
using c32 = float2;

// ---------------------------------------------------------------- device buffers
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevMem& operator=(DevMem&& o) noexcept {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    return *this;
  }
  ~DevMem();
  void alloc(size_t b);          // frees the old buffer, allocates b bytes (no-op when b fits)
  void ensure(size_t b);         // grows to at least b bytes
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory (hipHostMalloc): the source of host-to-device copies
// the host does not wait for.  ensure drops the old contents.
struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  HostPinned() = default;
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  ~HostPinned();
  void ensure(size_t b);  // grows to at least b bytes
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- FFT plans
constexpr int kMaxStages = 8;
struct FftPlan {
  int n = 0;
  int nst = 0;
  int radix[kMaxStages] = {0};
  int span[kMaxStages] = {0};  // product of the radices of the earlier stages
};
FftPlan make_plan(int n);      // radices from {4, 2, 3, 5}; fails for other primes

// ---------------------------------------------------------------- problem
struct KPoint {
  int64_t npw = 0;       // plane waves at this k
  int64_t off = 0;       // row offset in the stacked frame
  double k[3] = {0, 0, 0};
  double w = 0;
  std::vector<int> box;  // host copy of the linear box indices
  std::vector<int> plane_start;  // (ns + 1) row starts of each active i1 plane
  DevMem d_kin;          // double[npw] |k+G|^2/2
  DevMem d_kin32;        // float[npw]
  DevMem d_box;          // int[npw] linear box index
  DevMem d_plane_start;  // int[ns + 1]
};

struct Scalars;        // device scalar workspace (reductions)

struct Arena;  // defined in ops.h

struct Workspace {
  DevMem planes;       // T buffer: cols x ns x n2 x n3 complex (FP64 or FP32)
  DevMem grid_c;       // complex N_g scratch (potentials)
  DevMem partial;      // reduction partials
  DevMem small;        // small dense scratch
  DevMem gemm_part;    // split-K partials of the Gram kernels
  DevMem rho_part;     // per-column-group partial densities
  DevMem eig;          // scratch of the p x p eigensolver
  DevMem chol;         // scratch of the pivoted Cholesky
  DevMem f[10];        // frame-sized scratch used by the entry points and the solver
};

}  // namespace eahp

// Optional per-kernel timing with HIP events on the context stream.
// 0 inv_yz, 1 x_local, 2 fwd_yz, 3 x_density; 4..6 the same in FP32; 7 the
// L2-resident reduction of the projected FOM systems (q > 512);
// complex products (the "bytes" field counts flops, 8 per complex multiply-add):
// 8 A^H B FP64, 9 A M FP64, 10 A^H B FP32, 11 A M FP32 over n >= 1024 rows,
// 12..15 the same over fewer rows
constexpr int kProfKernels = 16;
constexpr int kProfGemm = 8;
constexpr int kProfTridiag = 7;
struct ProfSlot {
  std::vector<hipEvent_t> start, stop;
  int used = 0;
  double bytes = 0;
};

struct eahp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool prof = false;
  ProfSlot slot[kProfKernels];
  // second stream and events of overlapped work, created on first use
  hipStream_t aux_stream = nullptr;
  hipEvent_t aux_ev[3] = {nullptr, nullptr, nullptr};
  eahp::DevMem aux_part;  // split-K partials of the products on the second stream
  ~eahp_ctx();
};

struct eahp_problem {
  eahp_ctx* ctx = nullptr;
  // system
  double lat[9];      // column-major lattice vectors
  double B[9];        // reciprocal vectors as columns (a_i . b_j = 2 pi delta_ij)
  double Omega = 0;
  int natoms = 0;
  std::vector<double> R;  // natoms x 3 Cartesian positions
  std::vector<double> Z;
  double r_loc = 0.8, r_proj = 0.8, D_proj = 1.0, ecut = 0;
  int n[3] = {0, 0, 0};
  int m2max = 0;      // largest |m2| over the bases
  int64_t Ng = 0;
  int p = 0, nk = 0, precision = 0, terms = 15;
  double occ = 2.0;
  std::vector<eahp::KPoint> kp;
  int64_t ntot = 0;   // sum of npw
  int64_t nmax = 0;   // max npw
  // active x-planes (union over k), in ascending i1
  int ns = 0;
  std::vector<int> plane_i1;
  eahp::DevMem d_plane_i1;
  eahp::FftPlan plan[3];
  eahp::DevMem d_tw[3];    // z64 twiddles exp(-2 pi i m / n_d), m < n_d
  eahp::DevMem d_tw32[3];  // c32 twiddles
  // fields on the grid (double unless noted)
  eahp::DevMem d_vion, d_veff, d_veff32, d_rho, d_energy_dens;
  eahp::DevMem d_D;        // double[natoms] projector couplings
  // symmetry of a reduced k-set: the box partitioned into orbits of the operations
  int nsym = 0, norb = 0;
  eahp::DevMem d_orb_start;  // int[norb + 1]
  eahp::DevMem d_orb_idx;    // int[N_g] box indices, orbit by orbit
  // workspaces
  eahp::Workspace ws;
  eahp::Arena* arena = nullptr;  // solver-side buffers (retraction, transports, FOM), owned
  eahp::DevMem d_kdesc;     // KDesc[nk]
  eahp::DevMem d_krows;     // int64 (npw, off) per k: the ragged batch of the per-k products
  // projectors, stacked like a frame of natoms columns: the block of k-point
  // k (npw_k x natoms, column-major) starts at natoms * off_k
  eahp::DevMem d_proj;      // z64
  eahp::DevMem d_proj32;    // c32
  eahp::DevMem d_kw;        // double[nk]
  eahp::DevMem d_R;         // natoms x 3 positions (device)
  eahp::DevMem d_Zv;        // natoms charges (device)
  eahp::DevMem d_box;       // complex N_g scratch
  eahp::DevMem d_vals;      // per-column scratch (2 * nk * pmax doubles)
  eahp::DevMem d_scal;      // device scalar slots
  double* h_scal = nullptr; // pinned mirror of d_scal
  eahp::DevMem d_info;      // int status slots
  int* h_info = nullptr;
  // counters
  int64_t napply = 0, napply32 = 0;
  int fom_iters = 0;
  size_t footprint = 0;
  // frame H-applies captured as HIP graphs (eahp_problem_set_graphs): keyed by
  // the frame pointers and every workspace address the captured launches use
  struct HGraph {
    int seen = 0;
    hipGraphExec_t exec = nullptr;
  };
  bool graphs = false;
  std::map<std::array<uintptr_t, 8>, HGraph> hgraphs;
  int64_t graph_captures = 0, graph_replays = 0;
  void drop_graphs();
  ~eahp_problem();
};
