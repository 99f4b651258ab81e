// Crystal symmetry for symmetry-reduced k-point sets (Sec. 5.1: the number of
// k-points is the grid's k1 k2 k3 divided by the symmetries of the crystal).
//
// An operation (W, t) acts on fractional positions as x -> W x + t; W is an
// integer matrix with entries in {-1, 0, 1} that preserves the lattice metric
// A^T A, t in [0, 1)^3.  Only operations that map the FFT box onto itself are
// kept (W_ab != 0 only where n_a = n_b, n_a t_a an integer), so the density on
// the box is symmetrised exactly by an index permutation.  Rotations act on a
// fractional k-point as u -> W^T u; time reversal adds u -> -u.
//
// With a reduced k-set the density of the kept points is averaged over the
// operations, rho(i) <- |G|^-1 sum_g rho((W_g i + n t_g) mod n), before the
// potentials are formed; for a symmetric ground state this is the density of
// the full set, and the energy, potentials and H are those of the full set.
// As the operations form a group the average is the mean over the orbit of
// i, so the box is partitioned into orbits once, on the host, and the device
// pass reads and writes every box point once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "devcommon.h"
#include "kernels.h"
#include "ops.h"

namespace eahp {

namespace {

double det3i(const int* W) {
  return (double)W[0] * (W[4] * W[8] - W[5] * W[7]) - (double)W[1] * (W[3] * W[8] - W[5] * W[6]) +
         (double)W[2] * (W[3] * W[7] - W[4] * W[6]);
}

// Cartesian length of the fractional difference d modulo the lattice (L column-major).
double frac_dist(const double L[9], const double d[3]) {
  double e[3], s = 0.0;
  for (int i = 0; i < 3; ++i) e[i] = d[i] - std::nearbyint(d[i]);
  for (int i = 0; i < 3; ++i) {
    const double c = L[i] * e[0] + L[i + 3] * e[1] + L[i + 6] * e[2];
    s += c * c;
  }
  return std::sqrt(s);
}

bool box_compatible(const int* W, const int n[3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (W[3 * a + b] != 0 && n[a] != n[b]) return false;
  return true;
}

// Does (W, t) map every atom onto an atom of the same charge within tol (bohr)?
bool maps_atoms(const double L[9], int natoms, const double* frac, const double* Z, const int* W, const double t[3],
                double tol) {
  for (int a = 0; a < natoms; ++a) {
    double y[3];
    for (int i = 0; i < 3; ++i)
      y[i] = W[3 * i] * frac[3 * a] + W[3 * i + 1] * frac[3 * a + 1] + W[3 * i + 2] * frac[3 * a + 2] + t[i];
    bool hit = false;
    for (int b = 0; b < natoms && !hit; ++b) {
      if (Z[b] != Z[a]) continue;
      const double d[3] = {y[0] - frac[3 * b], y[1] - frac[3 * b + 1], y[2] - frac[3 * b + 2]};
      hit = frac_dist(L, d) <= tol;
    }
    if (!hit) return false;
  }
  return true;
}

// Fractional point u taken into [-tol, 1 - tol) per coordinate.
void wrap01(const double u[3], double v[3], double tol) {
  for (int i = 0; i < 3; ++i) {
    double x = u[i] - std::floor(u[i]);
    if (x >= 1.0 - tol) x -= 1.0;
    v[i] = x;
  }
}

// Lookup of fractional points modulo integers: cells of width 1e-6, neighbour
// cells searched so that points on a cell boundary are found.
struct PointIndex {
  static constexpr double kCell = 1e6;
  const double* pts;
  int np;
  double tol;
  std::unordered_map<uint64_t, std::vector<int>> cells;
  static uint64_t key(int64_t a, int64_t b, int64_t c) {
    return ((uint64_t)(a + (1 << 20)) << 42) | ((uint64_t)(b + (1 << 20)) << 21) | (uint64_t)(c + (1 << 20));
  }
  PointIndex(const double* p, int n, double t) : pts(p), np(n), tol(t) {
    for (int j = 0; j < n; ++j) {
      double v[3];
      wrap01(p + 3 * j, v, tol);
      cells[key((int64_t)std::floor(v[0] * kCell), (int64_t)std::floor(v[1] * kCell),
                (int64_t)std::floor(v[2] * kCell))]
          .push_back(j);
    }
  }
  int find(const double u[3]) const {
    double v[3];
    wrap01(u, v, tol);
    const int64_t c[3] = {(int64_t)std::floor(v[0] * kCell), (int64_t)std::floor(v[1] * kCell),
                          (int64_t)std::floor(v[2] * kCell)};
    int best = -1;
    for (int da = -1; da <= 1; ++da)
      for (int db = -1; db <= 1; ++db)
        for (int dc = -1; dc <= 1; ++dc) {
          auto it = cells.find(key(c[0] + da, c[1] + db, c[2] + dc));
          if (it == cells.end()) continue;
          for (int j : it->second) {
            bool same = true;
            for (int i = 0; i < 3 && same; ++i) {
              const double d = u[i] - pts[3 * j + i];
              same = std::fabs(d - std::nearbyint(d)) <= tol;
            }
            if (same && (best < 0 || j < best)) best = j;
          }
        }
    return best;
  }
};

}  // namespace

void find_symmetry(const eahp_system_desc* d, const int n[3], double symprec, std::vector<SymOp>& ops) {
  if (!(symprec > 0)) fail(EAHP_EINVAL, "symprec must be positive");
  if (d->natoms > 0 && (!d->frac || !d->Z)) fail(EAHP_EINVAL, "atoms without positions or charges");
  const double* L = d->lattice;
  double M[9], mmax = 0.0;  // metric A^T A
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int r = 0; r < 3; ++r) s += L[r + 3 * i] * L[r + 3 * j];
      M[3 * i + j] = s;
      mmax = std::max(mmax, std::fabs(s));
    }
  ops.clear();
  int W[9];
  for (int code = 0; code < 19683; ++code) {  // 3^9 matrices, entry order -1 < 0 < 1, first entry slowest
    int c = code;
    for (int e = 8; e >= 0; --e) {
      W[e] = c % 3 - 1;
      c /= 3;
    }
    if (std::fabs(std::fabs(det3i(W)) - 1.0) > 0.5) continue;
    bool metric = true;
    for (int i = 0; i < 3 && metric; ++i)
      for (int j = 0; j < 3 && metric; ++j) {
        double s = 0;  // (W^T M W)_ij
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s += W[3 * a + i] * M[3 * a + b] * W[3 * b + j];
        metric = std::fabs(s - M[3 * i + j]) <= 1e-8 * mmax;
      }
    if (!metric || !box_compatible(W, n)) continue;
    std::vector<std::array<double, 3>> found;
    const int ncand = d->natoms > 0 ? d->natoms : 1;
    for (int b = 0; b < ncand; ++b) {
      double t[3];
      if (d->natoms > 0) {
        if (d->Z[b] != d->Z[0]) continue;
        for (int i = 0; i < 3; ++i)
          t[i] = d->frac[3 * b + i] -
                 (W[3 * i] * d->frac[0] + W[3 * i + 1] * d->frac[1] + W[3 * i + 2] * d->frac[2]);
      } else {
        t[0] = t[1] = t[2] = 0.0;
      }
      bool grid = true;
      const int nmax = std::max(n[0], std::max(n[1], n[2]));
      for (int i = 0; i < 3; ++i) {
        t[i] -= std::floor(t[i]);
        const double nt = n[i] * t[i];
        if (std::fabs(nt - std::nearbyint(nt)) > 1e-6 * nmax) grid = false;
        t[i] = std::nearbyint(nt) / n[i];
        t[i] -= std::floor(t[i]);
      }
      if (!grid) continue;
      if (!maps_atoms(L, d->natoms, d->frac, d->Z, W, t, symprec)) continue;
      bool dup = false;
      for (const auto& s : found)
        dup = dup || (std::fabs(s[0] - t[0]) < 1e-12 && std::fabs(s[1] - t[1]) < 1e-12 && std::fabs(s[2] - t[2]) < 1e-12);
      if (!dup) found.push_back({t[0], t[1], t[2]});
    }
    std::sort(found.begin(), found.end());
    for (const auto& t : found) {
      SymOp o;
      std::memcpy(o.W, W, sizeof(W));
      for (int i = 0; i < 3; ++i) o.t[i] = t[i];
      ops.push_back(o);
    }
  }
}

void reduce_kpoints(int nrot_in, const int* rot, bool time_reversal, int nk, const double* kfrac, const double* kw,
                    std::vector<double>& kout, std::vector<double>& wout, std::vector<int>& owner) {
  const double tol = 1e-8;
  std::vector<std::array<int, 9>> rots;
  for (int g = 0; g < nrot_in; ++g) {
    std::array<int, 9> W;
    std::memcpy(W.data(), rot + 9 * g, sizeof(int) * 9);
    if (std::find(rots.begin(), rots.end(), W) == rots.end()) rots.push_back(W);
  }
  PointIndex index(kfrac, nk, tol);
  owner.assign(nk, -1);
  kout.clear();
  wout.clear();
  std::vector<int> members;
  for (int i = 0; i < nk; ++i) {
    if (owner[i] >= 0) continue;
    members.clear();
    const double* u = kfrac + 3 * i;
    for (const auto& W : rots)
      for (int s = 0; s < (time_reversal ? 2 : 1); ++s) {
        const double sg = s ? -1.0 : 1.0;
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = sg * (W[a] * u[0] + W[3 + a] * u[1] + W[6 + a] * u[2]);  // W^T u
        const int j = index.find(v);
        if (j < 0) fail(EAHP_EINVAL, "k-point " + std::to_string(i) + " maps outside the set");
        if (std::find(members.begin(), members.end(), j) == members.end()) members.push_back(j);
      }
    std::sort(members.begin(), members.end());
    const int idx = (int)wout.size();
    double w = 0.0;
    for (int j : members) {
      if (owner[j] >= 0 && owner[j] != idx) fail(EAHP_EINVAL, "the operations do not form a group on the k-set");
      owner[j] = idx;
      w += kw[j];
    }
    kout.insert(kout.end(), u, u + 3);
    wout.push_back(w);
  }
}

// ---------------------------------------------------------------- device side
// The operations form a group, so the average over them at a box point is the
// mean of the density over the point's orbit.  The orbits partition the box:
// one thread per orbit reads its members and writes the mean back in place.
__global__ void __launch_bounds__(256) k_orbit_mean(int norb, const int* __restrict__ start,
                                                     const int* __restrict__ idx, double* __restrict__ rho) {
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < norb; o += gridDim.x * blockDim.x) {
    const int b = start[o], e = start[o + 1];
    double s = 0.0;
    for (int j = b; j < e; ++j) s += rho[idx[j]];
    const double m = s / (double)(e - b);
    for (int j = b; j < e; ++j) rho[idx[j]] = m;
  }
}

void setup_symmetry(eahp_problem* pb, const eahp_system_desc* d) {
  pb->nsym = 0;
  pb->norb = 0;
  if (d->nsym < 0) fail(EAHP_EINVAL, "nsym must be >= 0");
  if (d->nsym <= 1) return;
  if (d->nsym > kMaxSymOps) fail(EAHP_EINVAL, "more than " + std::to_string(kMaxSymOps) + " symmetry operations");
  if (!d->sym_rot || !d->sym_trans) fail(EAHP_EINVAL, "symmetry operations without rotations or translations");
  const int ns = d->nsym;
  const int* n = pb->n;
  std::vector<std::array<int, 12>> tab(ns);  // W row-major, then the box shifts n_a t_a in [0, n_a)
  for (int g = 0; g < ns; ++g) {
    const int* W = d->sym_rot + 9 * g;
    for (int e = 0; e < 9; ++e)
      if (W[e] < -1 || W[e] > 1) fail(EAHP_EINVAL, "rotation entries must be -1, 0 or 1");
    if (std::fabs(std::fabs(det3i(W)) - 1.0) > 0.5) fail(EAHP_EINVAL, "rotation with determinant other than +-1");
    if (!box_compatible(W, n)) fail(EAHP_EINVAL, "operation does not map the FFT box onto itself");
    double t[3];
    for (int i = 0; i < 3; ++i) {
      const double nt = n[i] * d->sym_trans[3 * g + i];
      if (!(std::fabs(nt - std::nearbyint(nt)) <= 1e-6))
        fail(EAHP_EINVAL, "translation not commensurate with the FFT box");
      const int sh = (int)((std::llround(nt) % n[i] + n[i]) % n[i]);
      tab[g][9 + i] = sh;
      t[i] = (double)sh / n[i];
    }
    for (int e = 0; e < 9; ++e) tab[g][e] = W[e];
    if (!maps_atoms(d->lattice, d->natoms, d->frac, d->Z, W, t, 1e-4))
      fail(EAHP_EINVAL, "operation " + std::to_string(g) + " is not a symmetry of the crystal");
  }
  // closure: (W1, s1)(W2, s2) = (W1 W2, W1 s2 + s1) on the box
  std::vector<std::array<int, 12>> keys(tab);
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) fail(EAHP_EINVAL, "repeated symmetry operation");
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) {
      const int* A = tab[a].data();
      const int* Bo = tab[b].data();
      std::array<int, 12> c;
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
          c[3 * i + j] = A[3 * i] * Bo[j] + A[3 * i + 1] * Bo[3 + j] + A[3 * i + 2] * Bo[6 + j];
        int sh = (A[3 * i] * Bo[9] + A[3 * i + 1] * Bo[10] + A[3 * i + 2] * Bo[11] + A[9 + i]) % n[i];
        c[9 + i] = sh < 0 ? sh + n[i] : sh;
      }
      if (!std::binary_search(keys.begin(), keys.end(), c))
        fail(EAHP_EINVAL, "the symmetry operations do not form a group");
    }
  // orbits of the box points, members in the order they are reached
  const int64_t Ng = pb->Ng;
  std::vector<int> orbit_of(Ng, -1), start{0}, idx;
  idx.reserve(Ng);
  for (int64_t g = 0; g < Ng; ++g) {
    if (orbit_of[g] >= 0) continue;
    const int id = (int)start.size() - 1;
    const int i3 = (int)(g % n[2]), i2 = (int)((g / n[2]) % n[1]), i1 = (int)(g / ((int64_t)n[1] * n[2]));
    for (const auto& o : tab) {
      const int i[3] = {i1, i2, i3};
      int j[3];
      for (int a = 0; a < 3; ++a) {
        const int v = (o[3 * a] * i[0] + o[3 * a + 1] * i[1] + o[3 * a + 2] * i[2] + o[9 + a]) % n[a];
        j[a] = v < 0 ? v + n[a] : v;
      }
      const int64_t q = ((int64_t)j[0] * n[1] + j[1]) * n[2] + j[2];
      if (orbit_of[q] < 0) {
        orbit_of[q] = id;
        idx.push_back((int)q);
      }
    }
    start.push_back((int)idx.size());
  }
  pb->norb = (int)start.size() - 1;
  pb->d_orb_start.alloc(sizeof(int) * start.size());
  pb->d_orb_idx.alloc(sizeof(int) * idx.size());
  HIPCK(hipMemcpy(pb->d_orb_start.p, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(pb->d_orb_idx.p, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
  pb->nsym = ns;
}

void symmetrize_density(eahp_problem* pb) {
  if (pb->nsym <= 1) return;
  const int blocks = std::max(1, std::min((pb->norb + 255) / 256, 4096));
  hipLaunchKernelGGL(k_orbit_mean, dim3(blocks), dim3(256), 0, pb->ctx->stream, pb->norb, pb->d_orb_start.as<int>(),
                     pb->d_orb_idx.as<int>(), pb->d_rho.as<double>());
  HIPCK(hipGetLastError());
}

}  // namespace eahp
