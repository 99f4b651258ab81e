// Problem set-up (plane-wave bases, FFT plans, static fields) and the
// Kohn-Sham operators on frames: density, potentials, energy, H-apply,
// Lambda and residual.
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "ops.h"
#include "setup.h"

namespace eahp {

thread_local std::string g_last_error;

void fail(int status, const std::string& msg) { throw Error{status, msg}; }

void hip_check(hipError_t e, const char* what, int line) {
  if (e != hipSuccess) {
    fail(e == hipErrorOutOfMemory ? EAHP_ENOMEM : EAHP_EDEVICE,
         std::string(hipGetErrorString(e)) + " in " + what + " (line " + std::to_string(line) + ")");
  }
}

DevMem::~DevMem() {
  if (p) (void)hipFree(p);
}
void DevMem::alloc(size_t b) {
  if (p && b <= bytes) return;
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  if (b == 0) return;
  const hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    fail(EAHP_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
  }
  bytes = b;
}
void DevMem::ensure(size_t b) {
  if (b > bytes) alloc(b);
}

HostPinned::~HostPinned() {
  if (p) (void)hipHostFree(p);
}
void HostPinned::ensure(size_t b) {
  if (b <= bytes) return;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  bytes = 0;
  if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    fail(EAHP_ENOMEM, "hipHostMalloc of " + std::to_string(b) + " bytes failed");
  }
  bytes = b;
}

FftPlan make_plan(int n) {
  FftPlan P;
  P.n = n;
  int m = n, span = 1;
  auto push = [&](int r) {
    if (P.nst >= kMaxStages) fail(EAHP_EINVAL, "FFT length has too many factors");
    P.radix[P.nst] = r;
    P.span[P.nst] = span;
    span *= r;
    ++P.nst;
    m /= r;
  };
  while (m % 4 == 0) push(4);
  while (m % 2 == 0) push(2);
  while (m % 3 == 0) push(3);
  while (m % 5 == 0) push(5);
  if (m != 1) fail(EAHP_EINVAL, "FFT length " + std::to_string(n) + " is not 2/3/5-smooth");
  return P;
}

static int smooth_at_least(int nmin) {
  for (int n = std::max(nmin, 1);; ++n) {
    int m = n;
    for (int f : {2, 3, 5})
      while (m % f == 0) m /= f;
    if (m == 1) return n;
  }
}

static void inv3(const double* A, double* Ai) {  // column-major 3x3 inverse
  const double a = A[0], b = A[3], c = A[6], d = A[1], e = A[4], f = A[7], g = A[2], h = A[5], i = A[8];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  const double r[9] = {(e * i - f * h), -(d * i - f * g), (d * h - e * g),
                       -(b * i - c * h), (a * i - c * g), -(a * h - b * g),
                       (b * f - c * e), -(a * f - c * d), (a * e - b * d)};
  // r holds the cofactor matrix row-major as (row, col) = r[3*row + col]; inverse = cofactor^T / det
  for (int row = 0; row < 3; ++row)
    for (int col = 0; col < 3; ++col) Ai[row + 3 * col] = r[3 * col + row] / det;
}

static int freq_of(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// Plane waves of every k-point: G = B m with |k+G|^2/2 <= ecut, k = B kfrac.
// Also the largest |m_d| per direction (it fixes the smallest alias-free box).
void enumerate_bases(const eahp_system_desc* d, const double L[9], const double B[9],
                     std::vector<std::vector<std::array<int, 3>>>& ms, std::vector<std::vector<double>>& kins,
                     std::vector<std::array<double, 3>>& kvec, int mmax[3]) {
  const double gmax = std::sqrt(2.0 * d->ecut);
  ms.assign(d->nk, {});
  kins.assign(d->nk, {});
  kvec.assign(d->nk, {0.0, 0.0, 0.0});
  for (int ik = 0; ik < d->nk; ++ik) {
    double k[3];
    for (int i = 0; i < 3; ++i) {
      double s = 0;
      for (int j = 0; j < 3; ++j) s += B[i + 3 * j] * d->kfrac[3 * ik + j];
      k[i] = s;
      kvec[ik][i] = s;
    }
    const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    int lim[3];
    for (int dd = 0; dd < 3; ++dd) {
      // |m_d| <= |row d of B^-1| (gmax + |k|), B^-1 = L^T / (2 pi)
      const double rn = std::sqrt(L[0 + 3 * dd] * L[0 + 3 * dd] + L[1 + 3 * dd] * L[1 + 3 * dd] +
                                  L[2 + 3 * dd] * L[2 + 3 * dd]) / (2.0 * M_PI);
      lim[dd] = (int)std::ceil((gmax + kn) * rn) + 1;
    }
    for (int a = -lim[0]; a <= lim[0]; ++a)
      for (int b = -lim[1]; b <= lim[1]; ++b)
        for (int c = -lim[2]; c <= lim[2]; ++c) {
          double q[3];
          for (int i = 0; i < 3; ++i) q[i] = k[i] + B[i] * a + B[i + 3] * b + B[i + 6] * c;
          const double kin = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
          if (kin <= d->ecut) {
            ms[ik].push_back({a, b, c});
            kins[ik].push_back(kin);
            mmax[0] = std::max(mmax[0], std::abs(a));
            mmax[1] = std::max(mmax[1], std::abs(b));
            mmax[2] = std::max(mmax[2], std::abs(c));
          }
        }
  }
}

void reciprocal(const double L[9], double B[9]) {
  double Li[9];
  inv3(L, Li);
  // B = 2 pi L^-T: column j of B is row j of L^-1 times 2 pi
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) B[i + 3 * j] = 2.0 * M_PI * Li[j + 3 * i];
}

// Sizes of a system without touching the device: plane waves per k, the box,
// the number of active x-planes and an estimate of the device bytes a solve
// needs (frames of the solver and the entry points, the slab of a frame-wide
// H-apply, the block FOM with a Krylov basis of 8 p columns, grids).
void layout_estimate(const eahp_system_desc* d, std::vector<int64_t>& npw, int n[3], int& ns, size_t& bytes) {
  if (!d || d->nk <= 0 || d->p <= 0 || !(d->ecut > 0) || !d->kfrac || !d->kweight)
    fail(EAHP_EINVAL, "invalid system description");
  double B[9];
  reciprocal(d->lattice, B);
  std::vector<std::vector<std::array<int, 3>>> ms;
  std::vector<std::vector<double>> kins;
  std::vector<std::array<double, 3>> kvec;
  int mmax[3] = {0, 0, 0};
  enumerate_bases(d, d->lattice, B, ms, kins, kvec, mmax);
  for (int dd = 0; dd < 3; ++dd) n[dd] = d->fft[dd] > 0 ? d->fft[dd] : smooth_at_least(4 * mmax[dd] + 1);
  std::vector<char> used(n[0], 0);
  npw.assign(d->nk, 0);
  int64_t ntot = 0, nmax = 0;
  for (int ik = 0; ik < d->nk; ++ik) {
    npw[ik] = (int64_t)ms[ik].size();
    ntot += npw[ik];
    nmax = std::max(nmax, npw[ik]);
    for (const auto& m : ms[ik]) used[((m[0] % n[0]) + n[0]) % n[0]] = 1;
  }
  ns = 0;
  for (char u : used) ns += u;
  const double p = d->p, Ng = (double)n[0] * n[1] * n[2];
  const double ps = ((n[1] * n[2] + 15) / 16) * 16;
  const double frame = 16.0 * ntot * p;
  const double fom = 16.0 * nmax * (2.0 * 8 * p + 5 * p);
  const double slab = 16.0 * d->nk * p * ns * ps;
  const double grids = 16.0 * 12 * Ng + 24.0 * ntot * std::max(d->natoms, 1);
  bytes = (size_t)(30 * frame + fom + slab + grids + 64.0 * 1024 * 1024);
}

// -------------------------------------------------------------------- build
void build_problem(eahp_problem* pb, const eahp_system_desc* d) {
  if (!d || d->natoms < 0 || d->nk <= 0 || d->p <= 0 || !(d->ecut > 0) || !d->kfrac || !d->kweight)
    fail(EAHP_EINVAL, "invalid system description");
  if (d->natoms > 0 && (!d->frac || !d->Z)) fail(EAHP_EINVAL, "atoms without positions or charges");
  if (d->precision != EAHP_FP64 && d->precision != EAHP_MIXED) fail(EAHP_EINVAL, "unknown precision");
  hipStream_t st = pb->ctx->stream;
  std::memcpy(pb->lat, d->lattice, sizeof(pb->lat));
  reciprocal(pb->lat, pb->B);
  const double* L = pb->lat;
  pb->Omega = std::fabs(L[0] * (L[4] * L[8] - L[7] * L[5]) - L[3] * (L[1] * L[8] - L[7] * L[2]) +
                        L[6] * (L[1] * L[5] - L[4] * L[2]));
  pb->natoms = d->natoms;
  pb->R.assign(3 * d->natoms, 0.0);
  pb->Z.assign(d->Z, d->Z + d->natoms);
  for (int I = 0; I < d->natoms; ++I)
    for (int i = 0; i < 3; ++i) {
      double s = 0;
      for (int j = 0; j < 3; ++j) s += L[i + 3 * j] * d->frac[3 * I + j];
      pb->R[3 * I + i] = s;
    }
  pb->r_loc = d->r_loc;
  pb->r_proj = d->r_proj;
  pb->D_proj = d->D_proj;
  pb->ecut = d->ecut;
  pb->p = d->p;
  pb->nk = d->nk;
  pb->occ = d->occ;
  pb->precision = d->precision;
  pb->terms = d->terms;

  // ---- bases: |k+G|^2/2 <= ecut, G = B m
  std::vector<std::vector<std::array<int, 3>>> ms(d->nk);
  std::vector<std::vector<double>> kins(d->nk);
  int mmax[3] = {0, 0, 0};
  std::vector<std::array<double, 3>> kvec;
  enumerate_bases(d, pb->lat, pb->B, ms, kins, kvec, mmax);
  pb->kp.resize(d->nk);
  for (int ik = 0; ik < d->nk; ++ik) {
    auto& K = pb->kp[ik];
    for (int i = 0; i < 3; ++i) K.k[i] = kvec[ik][i];
    K.w = d->kweight[ik];
  }
  for (int dd = 0; dd < 3; ++dd) {
    pb->n[dd] = d->fft[dd] > 0 ? d->fft[dd] : smooth_at_least(4 * mmax[dd] + 1);
    if (2 * mmax[dd] >= pb->n[dd]) fail(EAHP_EINVAL, "FFT box too small for the basis");
  }
  pb->m2max = mmax[1];
  pb->Ng = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
  if (pb->Ng > INT32_MAX) fail(EAHP_EINVAL, "FFT box too large");
  setup_symmetry(pb, d);
  const int n1 = pb->n[0], n2 = pb->n[1], n3 = pb->n[2];
  std::vector<char> plane_used(n1, 0);
  pb->ntot = 0;
  pb->nmax = 0;
  for (int ik = 0; ik < d->nk; ++ik) {
    auto& K = pb->kp[ik];
    const size_t n = ms[ik].size();
    std::vector<std::pair<int, size_t>> order(n);
    for (size_t g = 0; g < n; ++g) {
      const auto& m = ms[ik][g];
      const int i1 = ((m[0] % n1) + n1) % n1, i2 = ((m[1] % n2) + n2) % n2, i3 = ((m[2] % n3) + n3) % n3;
      order[g] = {(i1 * n2 + i2) * n3 + i3, g};
      plane_used[i1] = 1;
    }
    std::sort(order.begin(), order.end());
    K.npw = (int64_t)n;
    K.off = pb->ntot;
    pb->ntot += K.npw;
    pb->nmax = std::max(pb->nmax, K.npw);
    K.box.resize(n);
    std::vector<double> kin(n);
    for (size_t g = 0; g < n; ++g) {
      K.box[g] = order[g].first;
      kin[g] = kins[ik][order[g].second];
    }
    std::vector<float> kin32(kin.begin(), kin.end());
    K.d_kin.alloc(sizeof(double) * std::max<size_t>(n, 1));
    K.d_kin32.alloc(sizeof(float) * std::max<size_t>(n, 1));
    K.d_box.alloc(sizeof(int) * std::max<size_t>(n, 1));
    HIPCK(hipMemcpy(K.d_kin.p, kin.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(K.d_kin32.p, kin32.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(K.d_box.p, K.box.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  }
  pb->plane_i1.clear();
  for (int i = 0; i < n1; ++i)
    if (plane_used[i]) pb->plane_i1.push_back(i);
  pb->ns = (int)pb->plane_i1.size();
  pb->d_plane_i1.alloc(sizeof(int) * pb->ns);
  HIPCK(hipMemcpy(pb->d_plane_i1.p, pb->plane_i1.data(), sizeof(int) * pb->ns, hipMemcpyHostToDevice));
  const int np = n2 * n3;
  for (auto& K : pb->kp) {
    K.plane_start.assign(pb->ns + 1, 0);
    size_t g = 0;
    for (int s = 0; s < pb->ns; ++s) {
      while (g < K.box.size() && K.box[g] / np < pb->plane_i1[s]) ++g;
      K.plane_start[s] = (int)g;
    }
    K.plane_start[pb->ns] = (int)K.box.size();
    K.d_plane_start.alloc(sizeof(int) * (pb->ns + 1));
    HIPCK(hipMemcpy(K.d_plane_start.p, K.plane_start.data(), sizeof(int) * (pb->ns + 1), hipMemcpyHostToDevice));
  }

  // ---- FFT plans and twiddles (FP64 cos/sin of 2 pi m / n)
  for (int dd = 0; dd < 3; ++dd) {
    const int n = pb->n[dd];
    pb->plan[dd] = make_plan(n);
    std::vector<z64> tw(n);
    std::vector<c32> tw32(n);
    for (int m = 0; m < n; ++m) {
      const double a = 2.0 * M_PI * (double)m / (double)n;
      tw[m].x = std::cos(a);
      tw[m].y = -std::sin(a);
      tw32[m].x = (float)tw[m].x;
      tw32[m].y = (float)tw[m].y;
    }
    pb->d_tw[dd].alloc(sizeof(z64) * n);
    pb->d_tw32[dd].alloc(sizeof(c32) * n);
    HIPCK(hipMemcpy(pb->d_tw[dd].p, tw.data(), sizeof(z64) * n, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(pb->d_tw32[dd].p, tw32.data(), sizeof(c32) * n, hipMemcpyHostToDevice));
  }

  // ---- static fields
  const int64_t Ng = pb->Ng;
  pb->d_vion.alloc(sizeof(double) * Ng);
  pb->d_veff.alloc(sizeof(double) * Ng);
  pb->d_veff32.alloc(sizeof(float) * Ng);
  pb->d_rho.alloc(sizeof(double) * Ng);
  pb->d_box.alloc(sizeof(z64) * Ng);
  pb->d_R.alloc(sizeof(double) * std::max(1, 3 * pb->natoms));
  pb->d_Zv.alloc(sizeof(double) * std::max(1, pb->natoms));
  pb->d_D.alloc(sizeof(double) * std::max(1, pb->natoms));
  if (pb->natoms) {
    std::vector<double> D(pb->natoms, pb->D_proj);
    HIPCK(hipMemcpy(pb->d_R.p, pb->R.data(), sizeof(double) * 3 * pb->natoms, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(pb->d_Zv.p, pb->Z.data(), sizeof(double) * pb->natoms, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(pb->d_D.p, D.data(), sizeof(double) * pb->natoms, hipMemcpyHostToDevice));
  }
  Lat lat;
  std::memcpy(lat.B, pb->B, sizeof(lat.B));
  if ((pb->terms & EAHP_TERM_ION) && pb->natoms) {
    launch_vion_g(st, n1, n2, n3, lat, pb->natoms, pb->d_R.as<double>(), pb->d_Zv.as<double>(), pb->r_loc, pb->Omega,
                  pb->d_box.as<z64>());
    const z64* tws[3] = {pb->d_tw[0].as<z64>(), pb->d_tw[1].as<z64>(), pb->d_tw[2].as<z64>()};
    launch_box_fft(st, n1, n2, n3, pb->plan, tws, pb->d_box.as<z64>(), 1.0);
    launch_real_part(st, Ng, pb->d_box.as<z64>(), 1.0, pb->d_vion.as<double>());
  } else {
    HIPCK(hipMemsetAsync(pb->d_vion.p, 0, sizeof(double) * Ng, st));
  }
  const bool nl = (pb->terms & EAHP_TERM_NONLOCAL) && pb->natoms > 0;
  std::vector<KDesc> kd(pb->nk);
  std::vector<double> kw(pb->nk);
  if (nl) {
    pb->d_proj.alloc(sizeof(z64) * pb->ntot * pb->natoms);
    pb->d_proj32.alloc(sizeof(c32) * pb->ntot * pb->natoms);
  }
  for (int ik = 0; ik < pb->nk; ++ik) {
    auto& K = pb->kp[ik];
    z64* P = nl ? pb->d_proj.as<z64>() + (int64_t)pb->natoms * K.off : nullptr;
    c32* P32 = nl ? pb->d_proj32.as<c32>() + (int64_t)pb->natoms * K.off : nullptr;
    if (nl)
      launch_projectors(st, K.npw, K.d_box.as<int>(), n1, n2, n3, lat, K.k, pb->natoms, pb->d_R.as<double>(),
                        pb->r_proj, pb->Omega, P, P32);
    kd[ik] = KDesc{K.npw, K.off, K.d_box.as<int>(), K.d_plane_start.as<int>(), K.d_kin.as<double>(),
                   K.d_kin32.as<float>(), P, P32, K.w};
    kw[ik] = K.w;
  }
  pb->d_kdesc.alloc(sizeof(KDesc) * pb->nk);
  pb->d_kw.alloc(sizeof(double) * pb->nk);
  std::vector<int64_t> krows(2 * (size_t)pb->nk);
  for (int ik = 0; ik < pb->nk; ++ik) {
    krows[2 * ik] = pb->kp[ik].npw;
    krows[2 * ik + 1] = pb->kp[ik].off;
  }
  pb->d_krows.alloc(sizeof(int64_t) * krows.size());
  HIPCK(hipMemcpy(pb->d_krows.p, krows.data(), sizeof(int64_t) * krows.size(), hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(pb->d_kdesc.p, kd.data(), sizeof(KDesc) * pb->nk, hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(pb->d_kw.p, kw.data(), sizeof(double) * pb->nk, hipMemcpyHostToDevice));
  pb->d_vals.alloc(sizeof(double) * 2 * pb->nk * std::max(pb->p, 64) * 8);
  pb->d_scal.alloc(sizeof(double) * kNumScal);
  HIPCK(hipHostMalloc((void**)&pb->h_scal, sizeof(double) * kNumScal, hipHostMallocDefault));
  pb->d_info.alloc(sizeof(int) * 1024);
  HIPCK(hipHostMalloc((void**)&pb->h_info, sizeof(int) * 1024, hipHostMallocDefault));
  HIPCK(hipStreamSynchronize(st));
}

// -------------------------------------------------------------------- helpers
// slab planes start on 256-byte boundaries (FP64) so every x-line tile is whole cache lines
int plane_stride(const eahp_problem* pb) { return ((pb->n[1] * pb->n[2] + 15) / 16) * 16; }
GridGeom geom(const eahp_problem* pb) {
  return GridGeom{pb->n[0], pb->n[1], pb->n[2], pb->ns, pb->d_plane_i1.as<int>(), plane_stride(pb), pb->m2max};
}

ColMap frame_map(const eahp_problem* pb) { return ColMap{pb->d_kdesc.as<KDesc>(), 0, pb->p, 1}; }
ColMap block_map(const eahp_problem* pb, int k, int ncols) { return ColMap{pb->d_kdesc.as<KDesc>(), k, ncols, 0}; }

template <typename T> void* planes_for(eahp_problem* pb, int ncols) {
  const size_t b = sizeof(cplx<T>) * (size_t)ncols * pb->ns * plane_stride(pb);
  pb->ws.planes.ensure(b);
  return pb->ws.planes.p;
}

void fetch_scalars(eahp_problem* pb, int n) {
  hipStream_t st = pb->ctx->stream;
  HIPCK(hipMemcpyAsync(pb->h_scal, pb->d_scal.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
}

double* scal(eahp_problem* pb, int i) { return pb->d_scal.as<double>() + i; }

// -------------------------------------------------------------------- kernel timing
// the context whose timing is on (for the products, which see only a stream)
std::atomic<eahp_ctx*> g_prof_ctx{nullptr};

static void slot_begin(eahp_ctx* c, int id) {
  ProfSlot& s = c->slot[id];
  if (s.used == (int)s.start.size()) {
    hipEvent_t a, b;
    HIPCK(hipEventCreate(&a));
    HIPCK(hipEventCreate(&b));
    s.start.push_back(a);
    s.stop.push_back(b);
  }
  HIPCK(hipEventRecord(s.start[s.used], c->stream));
}
void gemm_prof_begin(hipStream_t st, int slot) {
  eahp_ctx* c = g_prof_ctx.load();
  if (c && c->prof && c->stream == st) slot_begin(c, slot);
}
void gemm_prof_end(hipStream_t st, int slot, double flops) {
  eahp_ctx* c = g_prof_ctx.load();
  if (!c || !c->prof || c->stream != st) return;
  ProfSlot& s = c->slot[slot];
  HIPCK(hipEventRecord(s.stop[s.used], c->stream));
  ++s.used;
  s.bytes += flops;
}

void prof_begin(eahp_problem* pb, int id) {
  eahp_ctx* c = pb->ctx;
  if (!c->prof) return;
  ProfSlot& s = c->slot[id];
  if (s.used == (int)s.start.size()) {
    hipEvent_t a, b;
    HIPCK(hipEventCreate(&a));
    HIPCK(hipEventCreate(&b));
    s.start.push_back(a);
    s.stop.push_back(b);
  }
  HIPCK(hipEventRecord(s.start[s.used], c->stream));
}
void prof_end(eahp_problem* pb, int id, double bytes) {
  eahp_ctx* c = pb->ctx;
  if (!c->prof) return;
  ProfSlot& s = c->slot[id];
  HIPCK(hipEventRecord(s.stop[s.used], c->stream));
  ++s.used;
  s.bytes += bytes;
}
// algorithmic bytes of the three H-apply kernels and the density kernel for
// ncols columns whose plane-wave counts sum to npw_sum (b = bytes per complex)
static double bytes_inv(const eahp_problem* pb, int ncols, double npw_sum, int b) {
  return b * (npw_sum + (double)ncols * pb->ns * pb->n[1] * pb->n[2]);
}
static double bytes_xloc(const eahp_problem* pb, int ncols, int b) {
  return 2.0 * b * ncols * pb->ns * pb->n[1] * pb->n[2] + (b / 2) * (double)pb->Ng;
}
static double bytes_fwd(const eahp_problem* pb, int ncols, double npw_sum, int b) {
  return b * ((double)ncols * pb->ns * pb->n[1] * pb->n[2] + 2.0 * npw_sum) + (b / 2) * npw_sum;
}
static double bytes_dens(const eahp_problem* pb, int ncols) {
  return 16.0 * ncols * pb->ns * pb->n[1] * pb->n[2] + 8.0 * pb->Ng;
}

// -------------------------------------------------------------------- density and potentials
void potentials(eahp_problem* pb) {
  hipStream_t st = pb->ctx->stream;
  const int n1 = pb->n[0], n2 = pb->n[1], n3 = pb->n[2];
  const int64_t Ng = pb->Ng;
  z64* box = pb->d_box.as<z64>();
  const z64* tws[3] = {pb->d_tw[0].as<z64>(), pb->d_tw[1].as<z64>(), pb->d_tw[2].as<z64>()};
  if (pb->terms & EAHP_TERM_HARTREE) {
    launch_rho_to_box(st, Ng, pb->d_rho.as<double>(), box);
    launch_box_fft(st, n1, n2, n3, pb->plan, tws, box, -1.0);
    launch_hartree_g(st, n1, n2, n3, pb->B, box);
    launch_box_fft(st, n1, n2, n3, pb->plan, tws, box, 1.0);
  }
  const int nblk = 1024;
  pb->ws.partial.ensure(sizeof(double) * 3 * nblk);
  launch_veff(st, Ng, pb->d_rho.as<double>(), pb->d_vion.as<double>(), box, pb->terms, pb->d_veff.as<double>(),
              pb->d_veff32.as<float>(), pb->ws.partial.as<double>(), nblk);
  const double dv = pb->Omega / (double)Ng;
  for (int c = 0; c < 3; ++c) sum_strided(st, nblk, 3, c, pb->ws.partial.as<double>(), dv, scal(pb, S_ION + c));
}

// Inverse transforms of all frame columns into the plane buffer, density, potentials.
void density_potentials(eahp_problem* pb, const z64* Psi) {
  hipStream_t st = pb->ctx->stream;
  const int ncols = pb->nk * pb->p;
  z64* Tb = (z64*)planes_for<double>(pb, ncols);
  const GridGeom g = geom(pb);
  const double nsum = (double)pb->ntot * pb->p;
  prof_begin(pb, 0);
  launch_inv_yz<double>(st, frame_map(pb), ncols, g, pb->plan[2], pb->plan[1], pb->d_tw[2].as<z64>(),
                        pb->d_tw[1].as<z64>(), Psi, Tb);
  prof_end(pb, 0, bytes_inv(pb, ncols, nsum, 16));
  prof_begin(pb, 3);
  launch_x_density(st, frame_map(pb), ncols, g, pb->plan[0], pb->d_tw[0].as<z64>(), Tb, pb->occ / pb->Omega,
                   pb->d_rho.as<double>(), 0, pb->ws.rho_part);
  prof_end(pb, 3, bytes_dens(pb, ncols));
  symmetrize_density(pb);
  potentials(pb);
}

// -------------------------------------------------------------------- H-apply
// Stacked projectors (the block of k-point k at natoms off_k), and those of
// k-point ik (npw_k x natoms, leading dimension npw_k).
template <typename T>
const cplx<T>* proj_stack(const eahp_problem* pb) {
  if constexpr (sizeof(T) == 8) return pb->d_proj.as<z64>();
  else return pb->d_proj32.as<c32>();
}
template <typename T>
const cplx<T>* projectors(const eahp_problem* pb, int ik) {
  return proj_stack<T>(pb) + (int64_t)pb->natoms * pb->kp[ik].off;
}

// Nonlocal part on one k-block: HX += P (D (P^H X)); optional (FP64) per-column
// sum_I D_I |<beta_I, x_j>|^2 into nlvals.
template <typename T>
void nonlocal_block(eahp_problem* pb, int ik, int ncols, const cplx<T>* X, int64_t ldx, cplx<T>* HX, int64_t ldh,
                    double* nlvals) {
  if (!((pb->terms & EAHP_TERM_NONLOCAL) && pb->natoms > 0) || ncols <= 0) return;
  hipStream_t st = pb->ctx->stream;
  const int64_t n = pb->kp[ik].npw;
  const int na = pb->natoms;
  const cplx<T>* P = projectors<T>(pb, ik);
  pb->ws.small.ensure(sizeof(cplx<T>) * (size_t)na * ncols);
  cplx<T>* Bm = pb->ws.small.as<cplx<T>>();
  gemm_hn<T>(st, n, na, ncols, P, n, X, ldx, Bm, na, 1.0, 0.0, pb->ws.gemm_part);
  if constexpr (sizeof(T) == 8) {
    if (nlvals) col_weighted_norm2(st, na, ncols, Bm, na, pb->d_D.as<double>(), nlvals);
  }
  scale_rows<T>(st, na, ncols, pb->d_D.as<double>(), Bm, na);
  gemm_nn<T>(st, n, na, ncols, P, n, Bm, na, 0, HX, ldh, 1.0, 0.0, 1.0);
}

// The same for the k-points of a ragged batch (nb entries of ncols columns;
// X and HX stacked like a frame of ncols columns, or padded at kstride with
// leading dimension ld; rsum: the rows of all entries): three launches for
// all of them.  nlvals: entry b's columns at b ncols.
template <typename T>
void nonlocal_ragged(eahp_problem* pb, const Ragged& rg, int nb, int64_t rsum, int ncols, const cplx<T>* X,
                     int64_t ld, int64_t kstride, cplx<T>* HX, double* nlvals) {
  if (!((pb->terms & EAHP_TERM_NONLOCAL) && pb->natoms > 0) || ncols <= 0 || nb <= 0) return;
  hipStream_t st = pb->ctx->stream;
  const int na = pb->natoms;
  const cplx<T>* P = proj_stack<T>(pb);
  const int64_t sBm = (int64_t)na * ncols;
  pb->ws.small.ensure(sizeof(cplx<T>) * (size_t)sBm * nb);
  cplx<T>* Bm = pb->ws.small.as<cplx<T>>();
  gemm_hn_ragged<T>(st, rg, pb->nmax, rsum, na, ncols, P, X, ld, kstride, Bm, na, sBm, 1.0, 0.0, pb->ws.gemm_part,
                    nb);
  if constexpr (sizeof(T) == 8) {
    if (nlvals) col_weighted_norm2(st, na, ncols * nb, Bm, na, pb->d_D.as<double>(), nlvals);
  }
  scale_rows<T>(st, na, ncols * nb, pb->d_D.as<double>(), Bm, na);
  gemm_nn_ragged<T>(st, rg, pb->nmax, rsum, na, ncols, P, Bm, na, sBm, 0, HX, ld, kstride, 1.0, 1.0, nb);
}

// H X for a whole frame with the current V_eff.  tb_ready: the plane buffer
// already holds the inverse y/z transforms of X (from density_potentials).
static void apply_H_frame_launches(eahp_problem* pb, const z64* X, z64* HX, bool tb_ready, double* nlvals) {
  hipStream_t st = pb->ctx->stream;
  const int ncols = pb->nk * pb->p;
  z64* Tb = (z64*)planes_for<double>(pb, ncols);
  const GridGeom g = geom(pb);
  const ColMap cm = frame_map(pb);
  const double nsum = (double)pb->ntot * pb->p;
  if (!tb_ready) {
    prof_begin(pb, 0);
    launch_inv_yz<double>(st, cm, ncols, g, pb->plan[2], pb->plan[1], pb->d_tw[2].as<z64>(), pb->d_tw[1].as<z64>(),
                          X, Tb);
    prof_end(pb, 0, bytes_inv(pb, ncols, nsum, 16));
  }
  prof_begin(pb, 1);
  launch_x_local<double>(st, ncols, g, pb->plan[0], pb->d_tw[0].as<z64>(), pb->d_veff.as<double>(), Tb);
  prof_end(pb, 1, bytes_xloc(pb, ncols, 16));
  prof_begin(pb, 2);
  launch_fwd_yz<double>(st, cm, ncols, g, pb->plan[2], pb->plan[1], pb->d_tw[2].as<z64>(), pb->d_tw[1].as<z64>(), Tb,
                        X, HX);
  prof_end(pb, 2, bytes_fwd(pb, ncols, nsum, 16));
  if (pb->nk == 1) {
    nonlocal_block<double>(pb, 0, pb->p, X, pb->kp[0].npw, HX, pb->kp[0].npw, nlvals);
  } else {
    const Ragged rg{pb->d_krows.as<int64_t>(), nullptr, 1};
    nonlocal_ragged<double>(pb, rg, pb->nk, pb->ntot, pb->p, X, 0, 0, HX, nlvals);
  }
}

// With graphs on, the launch sequence of a frame H-apply is captured into a
// HIP graph the second time the same key occurs (the first call runs the
// launches directly and sizes every workspace they use), and replayed from
// then on.  The key holds the frame pointers and the addresses of the
// workspaces the captured kernels read and write, so a workspace that has
// been reallocated since leads to a new capture rather than a replay.  The
// graph takes the pointers, not the values: V_eff, the frames and the
// workspaces are read at replay time.  No memset is captured.  Kernel timing
// (eahp_prof_enable) runs the launches directly.
void apply_H_frame(eahp_problem* pb, const z64* X, z64* HX, bool tb_ready, double* nlvals) {
  hipStream_t st = pb->ctx->stream;
  const int ncols = pb->nk * pb->p;
  const bool use = pb->graphs && st != nullptr && !pb->ctx->prof && g_prof_ctx.load() == nullptr;
  if (!use) {
    apply_H_frame_launches(pb, X, HX, tb_ready, nlvals);
    pb->napply += ncols;
    return;
  }
  z64* Tb = (z64*)planes_for<double>(pb, ncols);
  const std::array<uintptr_t, 8> key = {(uintptr_t)X, (uintptr_t)HX, (uintptr_t)nlvals, (uintptr_t)tb_ready,
                                        (uintptr_t)Tb, (uintptr_t)pb->ws.small.p, (uintptr_t)pb->ws.gemm_part.p,
                                        (uintptr_t)pb->d_veff.p};
  auto& e = pb->hgraphs[key];
  if (e.exec) {
    HIPCK(hipGraphLaunch(e.exec, st));
    ++pb->graph_replays;
  } else if (e.seen == 0) {
    e.seen = 1;
    apply_H_frame_launches(pb, X, HX, tb_ready, nlvals);
  } else {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCK(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) {  // the caller is capturing: plain launches into its graph
      apply_H_frame_launches(pb, X, HX, tb_ready, nlvals);
    } else {
      HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      try {
        apply_H_frame_launches(pb, X, HX, tb_ready, nlvals);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hipGraph_t g = nullptr;
      HIPCK(hipStreamEndCapture(st, &g));
      const hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCK(ie);
      ++pb->graph_captures;
      HIPCK(hipGraphLaunch(e.exec, st));
      ++pb->graph_replays;
    }
  }
  pb->napply += ncols;
}

// H X for ncols columns of one k-block (ld = npw of that k).
template <typename T>
void apply_H_block(eahp_problem* pb, int ik, int ncols, const cplx<T>* X, cplx<T>* HX) {
  if (ncols <= 0) return;
  hipStream_t st = pb->ctx->stream;
  cplx<T>* Tb = (cplx<T>*)planes_for<T>(pb, ncols);
  const GridGeom g = geom(pb);
  const ColMap cm = block_map(pb, ik, ncols);
  const cplx<T>* twz = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[2].p : (const cplx<T>*)pb->d_tw32[2].p;
  const cplx<T>* twy = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[1].p : (const cplx<T>*)pb->d_tw32[1].p;
  const cplx<T>* twx = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[0].p : (const cplx<T>*)pb->d_tw32[0].p;
  const T* V = sizeof(T) == 8 ? (const T*)pb->d_veff.p : (const T*)pb->d_veff32.p;
  const double nsum = (double)pb->kp[ik].npw * ncols;
  const int b = 2 * (int)sizeof(T);
  const int slot0 = sizeof(T) == 8 ? 0 : 4;  // timing slots 4..7 hold the single-precision launches
  prof_begin(pb, slot0 + 0);
  launch_inv_yz<T>(st, cm, ncols, g, pb->plan[2], pb->plan[1], twz, twy, X, Tb);
  prof_end(pb, slot0 + 0, bytes_inv(pb, ncols, nsum, b));
  prof_begin(pb, slot0 + 1);
  launch_x_local<T>(st, ncols, g, pb->plan[0], twx, V, Tb);
  prof_end(pb, slot0 + 1, bytes_xloc(pb, ncols, b));
  prof_begin(pb, slot0 + 2);
  launch_fwd_yz<T>(st, cm, ncols, g, pb->plan[2], pb->plan[1], twz, twy, Tb, X, HX);
  prof_end(pb, slot0 + 2, bytes_fwd(pb, ncols, nsum, b));
  const int64_t n = pb->kp[ik].npw;
  nonlocal_block<T>(pb, ik, ncols, X, n, HX, n, nullptr);
  pb->napply += ncols;
  if (sizeof(T) == 4) pb->napply32 += ncols;
}
template void apply_H_block<double>(eahp_problem*, int, int, const z64*, z64*);
template void apply_H_block<float>(eahp_problem*, int, int, const c32*, c32*);

// H X for cpk columns of each of the k-points listed in kmap_dev / kmap_host
// (nact of them) in a padded batch: the block of k-point k starts at
// k * kstride, every column has leading dimension ld (rows npw_k.. are not
// read, and not written in HX).  One launch per transform over all columns.
template <typename T>
void apply_H_padded(eahp_problem* pb, int nact, const int* kmap_dev, const int* kmap_host, int cpk, const cplx<T>* X,
                    cplx<T>* HX, int64_t ld, int64_t kstride) {
  const int ncols = nact * cpk;
  if (ncols <= 0) return;
  hipStream_t st = pb->ctx->stream;
  cplx<T>* Tb = (cplx<T>*)planes_for<T>(pb, ncols);
  const GridGeom g = geom(pb);
  ColMap cm{pb->d_kdesc.as<KDesc>(), 0, cpk, 2};
  cm.ld = ld;
  cm.kstride = kstride;
  cm.kmap = kmap_dev;
  const cplx<T>* twz = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[2].p : (const cplx<T>*)pb->d_tw32[2].p;
  const cplx<T>* twy = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[1].p : (const cplx<T>*)pb->d_tw32[1].p;
  const cplx<T>* twx = sizeof(T) == 8 ? (const cplx<T>*)pb->d_tw[0].p : (const cplx<T>*)pb->d_tw32[0].p;
  const T* V = sizeof(T) == 8 ? (const T*)pb->d_veff.p : (const T*)pb->d_veff32.p;
  double nsum = 0;
  for (int a = 0; a < nact; ++a) nsum += (double)pb->kp[kmap_host[a]].npw * cpk;
  const int b = 2 * (int)sizeof(T);
  const int slot0 = sizeof(T) == 8 ? 0 : 4;
  prof_begin(pb, slot0 + 0);
  launch_inv_yz<T>(st, cm, ncols, g, pb->plan[2], pb->plan[1], twz, twy, X, Tb);
  prof_end(pb, slot0 + 0, bytes_inv(pb, ncols, nsum, b));
  prof_begin(pb, slot0 + 1);
  launch_x_local<T>(st, ncols, g, pb->plan[0], twx, V, Tb);
  prof_end(pb, slot0 + 1, bytes_xloc(pb, ncols, b));
  prof_begin(pb, slot0 + 2);
  launch_fwd_yz<T>(st, cm, ncols, g, pb->plan[2], pb->plan[1], twz, twy, Tb, X, HX);
  prof_end(pb, slot0 + 2, bytes_fwd(pb, ncols, nsum, b));
  if (nact == 1) {
    const int ik = kmap_host[0];
    nonlocal_block<T>(pb, ik, cpk, X + (int64_t)ik * kstride, ld, HX + (int64_t)ik * kstride, ld, nullptr);
  } else {
    const Ragged rg{pb->d_krows.as<int64_t>(), kmap_dev, 0};
    nonlocal_ragged<T>(pb, rg, nact, (int64_t)(nsum / cpk), cpk, X, ld, kstride, HX, nullptr);
  }
  pb->napply += ncols;
  if (sizeof(T) == 4) pb->napply32 += ncols;
}
template void apply_H_padded<double>(eahp_problem*, int, const int*, const int*, int, const z64*, z64*, int64_t,
                                     int64_t);
template void apply_H_padded<float>(eahp_problem*, int, const int*, const int*, int, const c32*, c32*, int64_t,
                                    int64_t);

// -------------------------------------------------------------------- point evaluation
// Everything the method needs at a point Psi (orthonormal frame):
// density, V_eff, energy terms, H Psi, Lambda (Hermitised) and R = H Psi - Psi Lambda.
void evaluate_point(eahp_problem* pb, const z64* Psi, z64* HPsi, z64* R, z64* Lam, PointScalars* out) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  density_potentials(pb, Psi);
  double* vals = pb->d_vals.as<double>();
  double* kinv = vals;
  double* nlv = vals + (size_t)nk * p;
  apply_H_frame(pb, Psi, HPsi, true, nlv);
  frame_col_wnorm2(st, pb->d_kdesc.as<KDesc>(), nk, p, Psi, 1, kinv);
  weighted_sum(st, nk, p, kinv, pb->d_kw.as<double>(), pb->occ, scal(pb, S_KIN));
  if ((pb->terms & EAHP_TERM_NONLOCAL) && pb->natoms > 0)
    weighted_sum(st, nk, p, nlv, pb->d_kw.as<double>(), pb->occ, scal(pb, S_NL));
  else
    weighted_sum(st, 0, p, nlv, pb->d_kw.as<double>(), 0.0, scal(pb, S_NL));  // writes 0
  lambda_residual(pb, Psi, HPsi, R, Lam);
  dot_re(st, pb->ntot * p, R, R, scal(pb, S_RR), pb->ws.partial);
  fetch_scalars(pb, S_RR + 1);
  if (out) {
    const double* h = pb->h_scal;
    out->terms[0] = h[S_KIN];
    out->terms[1] = h[S_NL];
    out->terms[2] = h[S_ION];
    out->terms[3] = h[S_HART];
    out->terms[4] = h[S_XC];
    out->E = h[S_KIN] + h[S_NL] + h[S_ION] + h[S_HART] + h[S_XC];
    out->rnorm = std::sqrt(std::max(0.0, h[S_RR]));
    if (!std::isfinite(out->E) || !std::isfinite(out->rnorm)) fail(EAHP_ENONFINITE, "non-finite energy or residual");
  }
}

// Energy at Psi without an H-apply: density, V_eff and the local terms, the
// kinetic term from the coefficients and the nonlocal term from the projector
// products.  Leaves the inverse y/z transforms of Psi in the plane buffer, so
// that complete_point can follow without repeating them.
void evaluate_energy(eahp_problem* pb, const z64* Psi, PointScalars* out) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  density_potentials(pb, Psi);
  double* vals = pb->d_vals.as<double>();
  double* kinv = vals;
  double* nlv = vals + (size_t)nk * p;
  const bool nl = (pb->terms & EAHP_TERM_NONLOCAL) && pb->natoms > 0;
  frame_col_wnorm2(st, pb->d_kdesc.as<KDesc>(), nk, p, Psi, 1, kinv);
  if (nl) {
    // sum_I D_I |<beta_I, psi_j>|^2 per column, all k-points at once
    const int na = pb->natoms;
    pb->ws.small.ensure(sizeof(z64) * (size_t)na * p * nk);
    z64* Bm = pb->ws.small.as<z64>();
    if (nk == 1) {
      const int64_t n = pb->kp[0].npw;
      gemm_hn<double>(st, n, na, p, projectors<double>(pb, 0), n, Psi, n, Bm, na, 1.0, 0.0, pb->ws.gemm_part);
    } else {
      const Ragged rg{pb->d_krows.as<int64_t>(), nullptr, 1};
      gemm_hn_ragged<double>(st, rg, pb->nmax, pb->ntot, na, p, proj_stack<double>(pb), Psi, 0, 0, Bm, na,
                             (int64_t)na * p, 1.0, 0.0, pb->ws.gemm_part, nk);
    }
    col_weighted_norm2(st, na, p * nk, Bm, na, pb->d_D.as<double>(), nlv);
  }
  weighted_sum(st, nk, p, kinv, pb->d_kw.as<double>(), pb->occ, scal(pb, S_KIN));
  if (nl) weighted_sum(st, nk, p, nlv, pb->d_kw.as<double>(), pb->occ, scal(pb, S_NL));
  else weighted_sum(st, 0, p, nlv, pb->d_kw.as<double>(), 0.0, scal(pb, S_NL));  // writes 0
  fetch_scalars(pb, S_NL + 1);
  const double* h = pb->h_scal;
  out->terms[0] = h[S_KIN];
  out->terms[1] = h[S_NL];
  out->terms[2] = h[S_ION];
  out->terms[3] = h[S_HART];
  out->terms[4] = h[S_XC];
  out->E = h[S_KIN] + h[S_NL] + h[S_ION] + h[S_HART] + h[S_XC];
  out->rnorm = 0;
  if (!std::isfinite(out->E)) fail(EAHP_ENONFINITE, "non-finite energy");
}

// H Psi, Lambda, R and ||R||_F at the point whose energy evaluate_energy just
// computed (V_eff and the plane buffer are still those of Psi).
void complete_point(eahp_problem* pb, const z64* Psi, z64* HPsi, z64* R, z64* Lam, PointScalars* out) {
  hipStream_t st = pb->ctx->stream;
  apply_H_frame(pb, Psi, HPsi, true, nullptr);
  lambda_residual(pb, Psi, HPsi, R, Lam);
  dot_re(st, pb->ntot * pb->p, R, R, scal(pb, S_RR), pb->ws.partial);
  fetch_scalars(pb, S_RR + 1);
  out->rnorm = std::sqrt(std::max(0.0, pb->h_scal[S_RR]));
  if (!std::isfinite(out->rnorm)) fail(EAHP_ENONFINITE, "non-finite residual");
}

// sum_k w_k Re tr(A_k^H B_k)
double frame_dot_weighted(eahp_problem* pb, const z64* A, const z64* B) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p, nk = pb->nk;
  double* vals = pb->d_vals.as<double>();
  for (int ik = 0; ik < nk; ++ik) {
    const int64_t o = (int64_t)p * pb->kp[ik].off;
    dot_re(st, pb->kp[ik].npw * p, A + o, B + o, vals + ik, pb->ws.partial);
  }
  weighted_sum(st, nk, 1, vals, pb->d_kw.as<double>(), 1.0, scal(pb, S_DOT));
  fetch_scalars(pb, S_DOT + 1);
  return pb->h_scal[S_DOT];
}

// One k-point: the plain product.  Several: one ragged batch over the
// k-blocks (row counts and offsets in d_krows).
void frames_hn(eahp_problem* pb, const z64* A, const z64* B, z64* C) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p;
  if (pb->nk == 1) {
    const int64_t n = pb->kp[0].npw;
    gemm_hn<double>(st, n, p, p, A, n, B, n, C, p, 1.0, 0.0, pb->ws.gemm_part);
    return;
  }
  const Ragged rg{pb->d_krows.as<int64_t>(), nullptr, 1};
  gemm_hn_ragged<double>(st, rg, pb->nmax, pb->ntot, p, p, A, B, 0, 0, C, p, (int64_t)p * p, 1.0, 0.0,
                         pb->ws.gemm_part, pb->nk);
}

void frames_nn(eahp_problem* pb, const z64* A, const z64* M, int opM, z64* C, double alpha, double beta) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p;
  if (pb->nk == 1) {
    const int64_t n = pb->kp[0].npw;
    gemm_nn<double>(st, n, p, p, A, n, M, p, opM, C, n, alpha, 0.0, beta);
    return;
  }
  const Ragged rg{pb->d_krows.as<int64_t>(), nullptr, 1};
  gemm_nn_ragged<double>(st, rg, pb->nmax, pb->ntot, p, p, A, M, p, (int64_t)p * p, opM, C, 0, 0, alpha, beta,
                         pb->nk);
}

// Lambda_k = herm(Psi_k^H (H Psi)_k), R_k = (H Psi)_k - Psi_k Lambda_k
void lambda_residual(eahp_problem* pb, const z64* Psi, const z64* HPsi, z64* R, z64* Lam) {
  hipStream_t st = pb->ctx->stream;
  const int p = pb->p;
  const int64_t pp = (int64_t)p * p;
  frames_hn(pb, Psi, HPsi, Lam);
  hermitize(st, p, Lam, p, pp, pb->nk);
  if (R) {
    axpby<double>(st, pb->ntot * p, 1.0, HPsi, 0.0, R);
    frames_nn(pb, Psi, Lam, 0, R, -1.0, 1.0);
  }
}

double frame_dot(eahp_problem* pb, const z64* A, const z64* B) {
  dot_re(pb->ctx->stream, pb->ntot * pb->p, A, B, scal(pb, S_DOT), pb->ws.partial);
  fetch_scalars(pb, S_DOT + 1);
  return pb->h_scal[S_DOT];
}

}  // namespace eahp

eahp_ctx::~eahp_ctx() {
  for (auto& s : slot) {
    for (auto e : s.start) (void)hipEventDestroy(e);
    for (auto e : s.stop) (void)hipEventDestroy(e);
  }
  if (aux_stream) {
    (void)hipSetDevice(device);
    (void)hipStreamSynchronize(aux_stream);
    (void)hipStreamDestroy(aux_stream);
  }
  for (auto e : aux_ev)
    if (e) (void)hipEventDestroy(e);
}

void eahp_problem::drop_graphs() {
  for (auto& kv : hgraphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  hgraphs.clear();
}

eahp_problem::~eahp_problem() {
  drop_graphs();
  delete arena;
  if (h_scal) (void)hipHostFree(h_scal);
  if (h_info) (void)hipHostFree(h_info);
}
