// Hermitian eigendecomposition A = V diag(w) V^H for n <= 128, one work-group
// of 1024 threads per matrix (batch over blockIdx.x):
//
//  1. Householder reduction to real symmetric tridiagonal form, Q^H A Q = T,
//     with the matrix held in registers (thread t owns row t/8 and the 16
//     columns congruent to t mod 8); reflectors H_k = I - tau_k v_k v_k^H are
//     chosen so that every subdiagonal entry comes out real.
//  2. Cuppen's divide and conquer on T, bottom up from 1 x 1 blocks: each
//     merge solves the secular equation of a rank-one update of a diagonal
//     matrix (Gu and Eisenstat's eigenvectors from the Loewner formula, so
//     they are orthogonal to working precision), with deflation of tiny
//     components and of close pole pairs by Givens rotations.  Q of the
//     current blocks lives in LDS.
//  3. V = Q Z, applying the reflectors to the real eigenvector matrix Z of T.
//
// Eigenvalues ascending.  Global scratch per matrix: the reflectors (n x n
// complex + n).
#include "devcommon.h"
#include "kernels.h"

namespace eahp {

namespace {

constexpr int kDcMax = 128;
constexpr double kEps = 2.220446049250313e-16;

__device__ __forceinline__ z64 cmulz(z64 a, z64 b) { return mk<double>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ z64 conjz(z64 a) { return mk<double>(a.x, -a.y); }

struct DcShared {
  double* Qs;   // n x n, column-major (aliased by the tridiagonalisation and back-transform buffers)
  double *D, *dl, *zz, *rc, *rs, *tv, *zh, *nrm, *dd, *ee, *Uc;
  int *srt, *nd, *dfl, *ra, *rb, *org, *outk, *Km, *nrot, *ndf;
};

// One secular root of 1 + rho sum_j z_j^2 / (dK_j - lam) = 0 for the i-th
// interval, by the fixed-weight rational iteration of the two nearest poles,
// safeguarded by the bracket; the sums over j are split over the 8 lanes of
// the calling group.  Returns tau with lam = dK[org] + tau.
__device__ double secular_root(const double* dK, const double* zK, int K, double rho, int i, int lane8, int& org) {
  const bool last = i == K - 1;
  // sum over the 8 lanes of the group (DPP within quads, then across the two
  // quads of the 8 lanes; the 8 lanes of a group are active together)
  auto sum8 = [&](double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
  };
  double lo, hi;
  int o;
  if (!last) {
    const double mid = 0.5 * (dK[i + 1] - dK[i]);
    double s = 0.0;
    for (int j = lane8; j < K; j += 8) s += zK[j] * zK[j] / ((dK[j] - dK[i]) - mid);
    const double fm = 1.0 + rho * sum8(s);
    if (fm >= 0.0) {
      o = i;
      lo = 0.0;
      hi = mid;
    } else {
      o = i + 1;
      lo = -mid;
      hi = 0.0;
    }
  } else {
    double s = 0.0;
    for (int j = lane8; j < K; j += 8) s += zK[j] * zK[j];
    o = K - 1;
    lo = 0.0;
    hi = rho * sum8(s);
  }
  const double dO = dK[o];
  double t = 0.5 * (lo + hi);
  for (int it = 0; it < 60; ++it) {
    double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0;
    for (int j = lane8; j < K; j += 8) {
      const double r = 1.0 / ((dK[j] - dO) - t);
      const double w = zK[j] * zK[j] * r;
      if (j <= i) {
        ps += w;
        dps += w * r;
      } else {
        ph += w;
        dph += w * r;
      }
    }
    ps = rho * sum8(ps);
    dps = rho * sum8(dps);
    ph = rho * sum8(ph);
    dph = rho * sum8(dph);
    const double f = 1.0 + ps + ph;
    if (f < 0.0) lo = t;
    else hi = t;
    // stop once f is within its own rounding error (the bound used by LAPACK's
    // secular solvers) or the bracket has collapsed
    const double erretm = 8.0 * (ph - ps) + 2.0 + 3.0 * fabs(t) * (dps + dph);
    if (fabs(f) <= kEps * erretm || hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi))) break;
    const double DL = (dK[i] - dO) - t;
    double eta;
    bool have = false;
    if (!last) {
      const double DR = (dK[i + 1] - dO) - t;
      const double a = dps * DL * DL, b = dph * DR * DR;
      const double c = f - dps * DL - dph * DR;
      const double A = c, B = c * (DL + DR) + a + b, C = c * DL * DR + a * DR + b * DL;
      const double sq = sqrt(fmax(B * B - 4.0 * A * C, 0.0));
      // the root of the two-pole model inside (DL, DR), from the stable forms first
      auto consider = [&](double v) {
        if (!have && v > DL && v < DR) {
          eta = v;
          have = true;
        }
      };
      if (B + sq != 0.0) consider(2.0 * C / (B + sq));
      if (B - sq != 0.0) consider(2.0 * C / (B - sq));
      if (A != 0.0) {
        consider((B + sq) / (2.0 * A));
        consider((B - sq) / (2.0 * A));
      }
      if (!have) eta = -f / (dps + dph);
    } else {
      const double a = dps * DL * DL, c = f - dps * DL;
      eta = (c != 0.0) ? DL + a / c : -f / dps;
    }
    double tn = t + eta;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (tn == t || fabs(tn - t) <= kEps * fabs(t)) {
      t = tn;
      break;
    }
    t = tn;
  }
  org = o;
  return t;
}

}  // namespace

__global__ void __launch_bounds__(1024) k_heev_dc(int n, const z64* __restrict__ Ab, int64_t lda, int64_t sA,
                                                  double* __restrict__ wb, int64_t sw, z64* __restrict__ Vb,
                                                  int64_t ldv, int64_t sV, double* __restrict__ scrb, int64_t sscr) {
  extern __shared__ unsigned char smem_raw[];
  DcShared S;
  S.Qs = reinterpret_cast<double*>(smem_raw);
  double* p = S.Qs + kDcMax * kDcMax;
  S.D = p; p += kDcMax;
  S.dl = p; p += kDcMax;
  S.zz = p; p += kDcMax;
  S.rc = p; p += kDcMax;
  S.rs = p; p += kDcMax;
  S.tv = p; p += kDcMax;
  S.zh = p; p += kDcMax;
  S.nrm = p; p += kDcMax;
  S.dd = p; p += kDcMax;
  S.ee = p; p += kDcMax;
  S.Uc = p; p += 8 * kDcMax;
  int* ip = reinterpret_cast<int*>(p);
  S.srt = ip; ip += kDcMax;
  S.nd = ip; ip += kDcMax;
  S.dfl = ip; ip += kDcMax;
  S.ra = ip; ip += kDcMax;
  S.rb = ip; ip += kDcMax;
  S.org = ip; ip += kDcMax;
  S.outk = ip; ip += kDcMax;
  S.Km = ip; ip += kDcMax;
  S.nrot = ip; ip += kDcMax;
  S.ndf = ip; ip += kDcMax;

  const z64* A = Ab + blockIdx.x * sA;
  double* w = wb + blockIdx.x * sw;
  z64* V = Vb + blockIdx.x * sV;
  double* scr = scrb + blockIdx.x * sscr;
  z64* refl = reinterpret_cast<z64*>(scr);            // n x n: column k holds v_k (rows k+1..n-1)
  z64* rtau = refl + (int64_t)n * n;                   // n

  const int t = threadIdx.x;
  const int r = t >> 3, cg = t & 7;

  // ------------------------------------------------------------ 1. tridiagonal form
  {
    // per column k: xs = column k, vs = the reflector, ps = tau A v, ws =
    // p + alpha v (each double-buffered by the parity of k).  Waves 0 and 1
    // (the rows) form the reflector and alpha with DPP wave sums; a wave whose
    // eight rows all lie above the trailing block skips the products.
    z64* xsb = reinterpret_cast<z64*>(S.Qs);
    z64* vsb = xsb + 2 * kDcMax;
    z64* psb = vsb + 2 * kDcMax;
    z64* wsb = psb + 2 * kDcMax;
    z64* taus = wsb + 2 * kDcMax;  // 2
    const int lane = t & 63;
    const int wv = t >> 6;
    d16 ar, ai;  // row r, columns cg + 8 m
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int c = cg + 8 * m;
      z64 v = mk<double>(0.0, 0.0);
      if (r < n && c < n) {
        const z64 x = A[r + (int64_t)c * lda], y = A[c + (int64_t)r * lda];
        v = mk<double>(0.5 * (x.x + y.x), r == c ? 0.0 : 0.5 * (x.y - y.y));
      }
      ar[m] = v.x;
      ai[m] = v.y;
    }
    for (int k = 0; k < n - 1; ++k) {
      z64* xs = xsb + (k & 1) * kDcMax;
      z64* vs = vsb + (k & 1) * kDcMax;
      z64* ps = psb + (k & 1) * kDcMax;
      z64* ws = wsb + (k & 1) * kDcMax;
      const int km = __builtin_amdgcn_readfirstlane(k >> 3);
      if (r < n && cg == (k & 7)) xs[r] = mk<double>(ar[km], ai[km]);
      __syncthreads();
      // reflector H = I - tau v v^H with v_{k+1} = 1 that maps x[k+1:] to beta e_1
      // (beta real), in waves 0 and 1 (vs[t] for t < 128)
      if (t < kDcMax) {
        double sg = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          if (i >= k + 2 && i < n) sg += xs[i].x * xs[i].x + xs[i].y * xs[i].y;
        }
        sg = wave_allsum(sg);
        const z64 al = xs[k + 1];
        double beta;
        z64 tau, inv;
        if (sg == 0.0 && al.y == 0.0) {
          tau = mk<double>(0.0, 0.0);
          beta = al.x;
          inv = mk<double>(0.0, 0.0);
        } else {
          const double nrm = sqrt(al.x * al.x + al.y * al.y + sg);
          beta = al.x >= 0.0 ? -nrm : nrm;
          tau = mk<double>((beta - al.x) / beta, -al.y / beta);
          const double dx = al.x - beta, dy = al.y;
          const double m2 = dx * dx + dy * dy;
          inv = mk<double>(dx / m2, -dy / m2);
        }
        const z64 v = (t <= k || t >= n) ? mk<double>(0.0, 0.0) : t == k + 1 ? mk<double>(1.0, 0.0) : cmulz(xs[t], inv);
        vs[t] = v;
        if (t > k && t < n) refl[t + (int64_t)k * n] = v;
        if (t == 0) {
          taus[k & 1] = tau;
          rtau[k] = tau;
          S.ee[k] = beta;
          S.dd[k] = xs[k].x;
        }
      }
      __syncthreads();
      // rows of this wave in the trailing block at all (wave-uniform)
      const bool active = __builtin_amdgcn_readfirstlane((8 * wv + 7 > k) ? 1 : 0) != 0;
      // p_r = tau (A v)_r (8 lanes per row, DPP sums); v is zero at rows <= k
      if (active) {
        z64 sv = mk<double>(0.0, 0.0);
#pragma unroll
        for (int mb = 0; mb < 16; mb += 4) {
          z64 vw[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) vw[u] = vs[cg + 8 * (mb + u)];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mb + u;
            sv.x += ar[m] * vw[u].x - ai[m] * vw[u].y;
            sv.y += ar[m] * vw[u].y + ai[m] * vw[u].x;
          }
        }
        sv.x += dpp_f64<0xB1>(sv.x);
        sv.y += dpp_f64<0xB1>(sv.y);
        sv.x += dpp_f64<0x4E>(sv.x);
        sv.y += dpp_f64<0x4E>(sv.y);
        sv.x += dpp_f64<0x141>(sv.x);  // row_half_mirror: the other quad of the 8 lanes
        sv.y += dpp_f64<0x141>(sv.y);
        if (cg == 0) ps[r] = (r > k && r < n) ? cmulz(taus[k & 1], sv) : mk<double>(0.0, 0.0);
      } else if (cg == 0) {
        ps[r] = mk<double>(0.0, 0.0);
      }
      __syncthreads();
      // w = p + alpha v with alpha = -tau (p^H v) / 2, in waves 0 and 1
      if (t < kDcMax) {
        double dx = 0.0, dy = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          const z64 pi = ps[i], vi = vs[i];
          dx += pi.x * vi.x + pi.y * vi.y;
          dy += pi.x * vi.y - pi.y * vi.x;
        }
        dx = wave_allsum(dx);
        dy = wave_allsum(dy);
        const z64 al2 = cscale<double>(cmulz(taus[k & 1], mk<double>(dx, dy)), -0.5);
        ws[t] = cadd<double>(ps[t], cmulz(al2, vs[t]));
      }
      __syncthreads();
      // A -= v w^H + w v^H on the trailing block (v, w vanish outside rows and
      // columns > k, so the rows of an active wave need no branch)
      if (active) {
        const z64 vr = vs[r], wr = ws[r];
#pragma unroll
        for (int mb = 0; mb < 16; mb += 4) {
          z64 vw[4], ww[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            vw[u] = vs[cg + 8 * (mb + u)];
            ww[u] = ws[cg + 8 * (mb + u)];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int m = mb + u;
            const z64 vc = vw[u], wc = ww[u];
            // v_r conj(w_c) + w_r conj(v_c)
            ar[m] -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
            ai[m] -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
          }
        }
      }
    }
    if (r == n - 1 && cg == ((n - 1) & 7)) S.dd[n - 1] = ar[__builtin_amdgcn_readfirstlane((n - 1) >> 3)];
    __syncthreads();
  }

  // ------------------------------------------------------------ 2. divide and conquer on (dd, ee)
  double* Q = S.Qs;
  for (int e = t; e < n * n; e += blockDim.x) Q[e] = (e % n == e / n) ? 1.0 : 0.0;
  for (int i = t; i < n; i += blockDim.x) {
    double v = S.dd[i];
    if (i > 0) v -= fabs(S.ee[i - 1]);
    if (i < n - 1) v -= fabs(S.ee[i]);
    S.D[i] = v;
  }
  __syncthreads();
  for (int size = 1; size < n; size *= 2) {
    const int nmerge = (n + 2 * size - 1) / (2 * size);
    // A1: merge the two ascending halves of every block and gather z, one
    // thread per element: its output position is its index in its own half
    // plus the count of smaller entries of the other half (ties: left half first)
    for (int g = t; g < n; g += blockDim.x) {
      const int mi = g / (2 * size), s = mi * 2 * size;
      const int n1 = min(size, n - s), n2 = min(size, n - s - n1);
      if (n2 <= 0) continue;
      const int j = g - s;
      const double x = S.D[g];
      int lo, cnt;
      if (j < n1) {  // entries of the right half strictly below x
        lo = 0, cnt = n2;
        while (cnt > 0) {
          const int h = cnt >> 1;
          if (S.D[s + n1 + lo + h] < x) {
            lo += h + 1;
            cnt -= h + 1;
          } else {
            cnt = h;
          }
        }
      } else {  // entries of the left half at or below x
        lo = 0, cnt = n1;
        while (cnt > 0) {
          const int h = cnt >> 1;
          if (S.D[s + lo + h] <= x) {
            lo += h + 1;
            cnt -= h + 1;
          } else {
            cnt = h;
          }
        }
      }
      const int q = (j < n1 ? j : j - n1) + lo;
      const double ev = S.ee[s + n1 - 1];
      const double sg = ev >= 0.0 ? 1.0 : -1.0;
      S.srt[s + q] = j;
      S.dl[s + q] = x;
      S.zz[s + q] = (j < n1 ? Q[(s + n1 - 1) + (s + j) * n] : sg * Q[(s + n1) + (s + j) * n]) * 0.7071067811865476;
    }
    __syncthreads();
    // A2: deflate (one thread per merge)
    if (t < nmerge) {
      const int s = t * 2 * size;
      const int n1 = min(size, n - s), n2 = min(size, n - s - n1);
      S.Km[t] = 0;
      S.nrot[t] = 0;
      S.ndf[t] = 0;
      if (n2 > 0) {
        const int m = n1 + n2;
        const double ev = S.ee[s + n1 - 1];
        const double rho = 2.0 * fabs(ev);
        double dmax = 0.0, zmax = 0.0;
        for (int q = 0; q < m; ++q) {
          dmax = fmax(dmax, fabs(S.dl[s + q]));
          zmax = fmax(zmax, fabs(S.zz[s + q]));
        }
        const double tol = 8.0 * kEps * fmax(dmax, rho * zmax);
        int K = 0, nd = 0, nr = 0, pj = -1;
        for (int j = 0; j < m; ++j) {
          if (rho * fabs(S.zz[s + j]) <= tol) {
            S.dfl[s + nd++] = j;
            continue;
          }
          if (pj < 0) {
            pj = j;
            continue;
          }
          const double zs = S.zz[s + pj], zc = S.zz[s + j];
          const double tau = hypot(zc, zs);
          const double c = zc / tau, sn = -zs / tau;
          const double tt = S.dl[s + j] - S.dl[s + pj];
          if (fabs(tt * c * sn) <= tol) {
            S.zz[s + j] = tau;
            S.zz[s + pj] = 0.0;
            S.ra[s + nr] = S.srt[s + pj];
            S.rb[s + nr] = S.srt[s + j];
            S.rc[s + nr] = c;
            S.rs[s + nr] = sn;
            ++nr;
            const double dp = S.dl[s + pj], dj = S.dl[s + j];
            S.dl[s + pj] = c * c * dp + sn * sn * dj;
            S.dl[s + j] = sn * sn * dp + c * c * dj;
            S.dfl[s + nd++] = pj;
            pj = j;
          } else {
            S.nd[s + K++] = pj;
            pj = j;
          }
        }
        if (pj >= 0) S.nd[s + K++] = pj;
        S.Km[t] = K;
        S.nrot[t] = nr;
        S.ndf[t] = nd;
      }
    }
    __syncthreads();
    // B: the deflation rotations act on columns of the block's eigenvector matrix
    for (int R = t; R < n; R += blockDim.x) {
      const int mi = R / (2 * size), s = mi * 2 * size;
      const int nr = S.nrot[mi];
      for (int q = 0; q < nr; ++q) {
        const int ca = s + S.ra[s + q], cb = s + S.rb[s + q];
        const double c = S.rc[s + q], sn = S.rs[s + q];
        const double qa = Q[R + ca * n], qb = Q[R + cb * n];
        Q[R + ca * n] = c * qa + sn * qb;
        Q[R + cb * n] = -sn * qa + c * qb;
      }
    }
    // C: secular roots, 8 lanes per root (slot g = s + i);
    // gather the non-deflated poles/weights contiguously (dK into tv, zK into nrm)
    for (int g = t; g < n; g += blockDim.x) {
      const int mi = g / (2 * size), s = mi * 2 * size, i = g - s;
      if (i < S.Km[mi]) {
        S.tv[g] = S.dl[s + S.nd[s + i]];
        S.nrm[g] = S.zz[s + S.nd[s + i]];
      }
    }
    __syncthreads();
    // roots: lam_i = dK[org_i] + tau_i; origin index into org, tau into rc (rotations are done)
    {
      const int g = t >> 3, lane8 = t & 7;
      if (g < n) {
        const int mi = g / (2 * size), s = mi * 2 * size, i = g - s;
        const int K = S.Km[mi];
        if (i < K) {
          const double rho = 2.0 * fabs(S.ee[s + min(size, n - s) - 1]);
          int o;
          const double tau = secular_root(S.tv + s, S.nrm + s, K, rho, i, lane8, o);
          if (lane8 == 0) {
            S.org[g] = o;
            S.rc[g] = tau;
          }
        }
      }
    }
    __syncthreads();
    // The secular differences delta(root k, pole i) = dK_i - lambda_k are
    // formed where needed as (dK_i - dK_org(k)) - tau_k (the root relative to
    // its nearest pole, which keeps them accurate); U[i][k] = z^_i / delta(k, i).
    // E: Loewner weights z^_i (sign of z_i)
    for (int g = t; g < n; g += blockDim.x) {
      const int mi = g / (2 * size), s = mi * 2 * size, i = g - s;
      const int K = S.Km[mi];
      if (i < K) {
        const double* dK = S.tv + s;
        const double di = dK[i];
        double wv = (di - dK[S.org[g]]) - S.rc[g];
        for (int j = 0; j < K; ++j)
          if (j != i) wv *= ((di - dK[S.org[s + j]]) - S.rc[s + j]) / (di - dK[j]);
        S.zh[g] = copysign(sqrt(fmax(-wv, 0.0)), S.nrm[g]);
      }
    }
    __syncthreads();
    // F: column norms of U (8 lanes per column), the final order of each merged
    // block (one thread per merge) and the source columns of the product
    {
      const int g = t >> 3, lane8 = t & 7;
      double acc = 0.0;
      int K = 0, s = 0;
      if (g < n) {
        const int mi = g / (2 * size);
        s = mi * 2 * size;
        K = S.Km[mi];
        if (g - s < K) {
          const double lo = S.tv[s + S.org[g]], tk = S.rc[g];
          for (int i = lane8; i < K; i += 8) {
            const double u = S.zh[s + i] / ((S.tv[s + i] - lo) - tk);
            acc += u * u;
          }
        }
      }
      acc += dpp_f64<0xB1>(acc);
      acc += dpp_f64<0x4E>(acc);
      acc += dpp_f64<0x141>(acc);
      if (g < n && g - s < K && lane8 == 0) S.dd[g] = 1.0 / sqrt(acc);  // the diagonal of T is no longer needed
    }
    for (int g = t; g < n; g += blockDim.x) {
      const int mi = g / (2 * size), s = mi * 2 * size, i = g - s;
      if (i < S.Km[mi]) S.ra[g] = s + S.srt[s + S.nd[s + i]];  // Q column of non-deflated pole i
    }
    if (t < nmerge) {
      const int s = t * 2 * size;
      const int n1 = min(size, n - s), n2 = min(size, n - s - n1);
      if (n2 > 0) {
        const int m = n1 + n2, K = S.Km[t], nd = S.ndf[t];
        // insertion sort of the deflated values (ascending), stable
        for (int a2 = 1; a2 < nd; ++a2) {
          const int v = S.dfl[s + a2];
          const double key = S.dl[s + v];
          int b2 = a2 - 1;
          while (b2 >= 0 && S.dl[s + S.dfl[s + b2]] > key) {
            S.dfl[s + b2 + 1] = S.dfl[s + b2];
            --b2;
          }
          S.dfl[s + b2 + 1] = v;
        }
        // outk[q] >= 0: root outk[q]; otherwise the Q column -outk[q] - 1 (deflated);
        // rb[k] = output position of root k
        int ia = 0, ib = 0;
        for (int q = 0; q < m; ++q) {
          const double lr = ia < K ? S.tv[s + S.org[s + ia]] + S.rc[s + ia] : 0.0;
          const double ld = ib < nd ? S.dl[s + S.dfl[s + ib]] : 0.0;
          if (ib >= nd || (ia < K && lr <= ld)) {
            S.outk[s + q] = ia;
            S.rb[s + ia] = q;
            S.D[s + q] = lr;
            ++ia;
          } else {
            S.outk[s + q] = -(s + S.srt[s + S.dfl[s + ib]] + 1);
            S.D[s + q] = ld;
            ++ib;
          }
        }
      }
    }
    __syncthreads();
    // G: merged eigenvectors, Q[:, block] <- Q[:, ra] U diag(dd) with the roots
    // in output order and the deflated columns moved to theirs.  Thread (row R,
    // column group cgp) forms the roots k = cgp + 8 j of its block; rows of U
    // are computed into LDS 8 at a time.  Every thread reads only its own row
    // of Q, so after a barrier the results go straight back into Q.
    {
      const int R = t & (kDcMax - 1), cgp = t >> 7;
      int kmax = 0;
      for (int q = 0; q < nmerge; ++q) kmax = max(kmax, S.Km[q]);
      const int mi = R / (2 * size), s = mi * 2 * size;
      const int n1 = min(size, n - s), n2 = min(size, n - s - n1);
      const bool valid = R < n && n2 > 0;
      const int K = valid ? S.Km[mi] : 0;
      const int m = n1 + n2;
      double acc[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = 0.0;
      for (int i0 = 0; i0 < kmax; i0 += 8) {
        __syncthreads();
        {
          const int ii = t >> 7, C = t & (kDcMax - 1);
          double u = 0.0;
          if (C < n) {
            const int mc = C / (2 * size), sc = mc * 2 * size, Kc = S.Km[mc];
            const int i = i0 + ii;
            if (i < Kc && C - sc < Kc) u = S.zh[sc + i] / ((S.tv[sc + i] - S.tv[sc + S.org[C]]) - S.rc[C]);
          }
          S.Uc[ii * kDcMax + C] = u;
        }
        __syncthreads();
        if (valid) {
          for (int ii = 0; ii < 8 && i0 + ii < K; ++ii) {
            const double qv = Q[R + S.ra[s + i0 + ii] * n];
            const double* urow = S.Uc + ii * kDcMax + s;
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] += qv * urow[min(cgp + 8 * j, kDcMax - 1 - s)];
          }
        }
      }
      double dfv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int q = cgp + 8 * j;
        const int o = (valid && q < m) ? S.outk[s + q] : 0;
        dfv[j] = o < 0 ? Q[R + (-o - 1) * n] : 0.0;
      }
      __syncthreads();  // every row of Q has been read
      if (valid) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = cgp + 8 * j;
          if (k < K) Q[R + (s + S.rb[s + k]) * n] = acc[j] * S.dd[s + k];
          if (k < m && S.outk[s + k] < 0) Q[R + (s + k) * n] = dfv[j];
        }
      }
    }
    __syncthreads();
  }

  // ------------------------------------------------------------ 3. V = Q_householder Z
  {
    const int c = t >> 3, rg = t & 7;  // column c, rows rg + 8 m
    z64 zv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int rr = rg + 8 * m;
      zv[m] = mk<double>((c < n && rr < n) ? Q[rr + c * n] : 0.0, 0.0);
    }
    for (int i = t; i < n; i += blockDim.x) w[i] = S.D[i];
    __syncthreads();
    constexpr int CH = 32;
    z64* vst = reinterpret_cast<z64*>(S.Qs);  // CH x n reflectors
    z64* tst = vst + CH * kDcMax;              // CH taus
    for (int k1 = n - 2; k1 >= 0; k1 -= CH) {
      const int k0 = max(0, k1 - CH + 1);
      const int cnt = k1 - k0 + 1;
      for (int e = t; e < cnt * n; e += blockDim.x) {
        const int kk = e / n, i = e % n;
        const int k = k0 + kk;
        vst[kk * kDcMax + i] = i > k ? refl[i + (int64_t)k * n] : mk<double>(0.0, 0.0);
      }
      for (int kk = t; kk < cnt; kk += blockDim.x) tst[kk] = rtau[k0 + kk];
      __syncthreads();
      for (int k = k1; k >= k0; --k) {
        const z64* vk = vst + (k - k0) * kDcMax;
        const z64 tk = tst[k - k0];
        z64 s = mk<double>(0.0, 0.0);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int rr = rg + 8 * m;
          if (rr > k && rr < n) s = cadd<double>(s, cmulz(conjz(vk[rr]), zv[m]));
        }
        s.x += dpp_f64<0xB1>(s.x);  // sum over the 8 lanes of the column
        s.y += dpp_f64<0xB1>(s.y);
        s.x += dpp_f64<0x4E>(s.x);
        s.y += dpp_f64<0x4E>(s.y);
        s.x += dpp_f64<0x141>(s.x);
        s.y += dpp_f64<0x141>(s.y);
        const z64 f = cmulz(tk, s);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int rr = rg + 8 * m;
          if (rr > k && rr < n) zv[m] = csub<double>(zv[m], cmulz(f, vk[rr]));
        }
      }
      __syncthreads();
    }
    if (c < n) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int rr = rg + 8 * m;
        if (rr < n) V[rr + (int64_t)c * ldv] = zv[m];
      }
    }
  }
}

size_t heev_dc_scratch(int n) { return sizeof(z64) * ((size_t)n * n + n) + 256; }

static void heev_dc_raw(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V,
                        int64_t ldv, int64_t sV, int batch, double* scr) {
  const int64_t per = (int64_t)((heev_dc_scratch(n) + 255) / 256 * 256 / sizeof(double));
  const size_t lds = sizeof(double) * ((size_t)kDcMax * kDcMax + 18 * kDcMax) + sizeof(int) * 10 * kDcMax;
  HIPCK(hipFuncSetAttribute((const void*)k_heev_dc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_heev_dc, dim3(batch), dim3(1024), lds, st, n, A, lda, sA, w, sw, V, ldv, sV, scr, per);
  HIPCK(hipGetLastError());
}

bool heev_dc(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V, int64_t ldv,
             int64_t sV, int batch, DevMem& scr) {
  if (n < 1 || n > kDcMax) return false;
  const int64_t per = (int64_t)((heev_dc_scratch(n) + 255) / 256 * 256 / sizeof(double));
  scr.ensure(sizeof(double) * per * batch);
  heev_dc_raw(st, n, A, lda, sA, w, sw, V, ldv, sV, batch, scr.as<double>());
  return true;
}

// ===========================================================================
// Hermitian eigendecomposition for kDcMax < n <= kDcBig, one matrix at a time:
//
//  1. A = Q T Q^H by tridiag_reduce (Householder reflectors, several
//     work-groups); T Hermitian tridiagonal with T[k+1][k] = e_k.
//  2. Phases P_0 = 1, P_{k+1} = P_k e_k / |e_k|, so that P^H T P = R is real
//     symmetric tridiagonal with R[k+1][k] = |e_k| >= 0.
//  3. R is padded to N' = L mL (L a power of two, mL <= kDcMax) with
//     decoupled diagonal entries above its spectrum, torn at the L - 1 leaf
//     boundaries (Cuppen: the coupling |e| is subtracted from the two
//     diagonal entries beside a boundary and restored as a rank-one term),
//     and the L leaves are solved by k_heev_dc in one batched launch.
//  4. log2 L levels of merges, every merge of two blocks on the device in
//     global memory: the eigenvalues of diag(D1, D2) + rho z z^T with the
//     deflation rules of k_heev_dc, the roots of the secular equation, the
//     Gu-Eisenstat eigenvector matrix U (K x K, from the Loewner weights,
//     columns normalised) and the block's eigenvector columns times U (an FP64
//     product), into a second buffer (the blocks of a level cover it).
//  5. V = Q P Z, with Z the leading n x n part of the eigenvector matrix of
//     the padded R (the pad entries are exactly decoupled, so their
//     eigenvalues come last and Z vanishes in the pad rows).
// ===========================================================================
constexpr int kDcBig = 2048;

namespace {

struct DcBig {
  int n, N, L, mL;
  double *Rd, *Rb, *D, *dl, *zz, *tv, *nrm, *zh, *cn, *rc, *rs, *tau;
  int *srt, *nd, *dfl, *ra, *rb, *org, *outk, *src, *Km, *nrot, *ndf;
};

__global__ void k_dc_phase(int n, int N, const double* __restrict__ dd, const z64* __restrict__ e, z64* Ph,
                           double* Rd, double* Rb) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  z64 P = mk<double>(1.0, 0.0);
  double dmax = 0.0, bmax = 0.0;
  for (int k = 0; k < n; ++k) {
    Ph[k] = P;
    Rd[k] = dd[k];
    dmax = fmax(dmax, fabs(dd[k]));
    if (k + 1 < n) {
      const z64 ek = e[k];
      const double a = sqrt(ek.x * ek.x + ek.y * ek.y);
      Rb[k] = a;
      bmax = fmax(bmax, a);
      if (a > 0.0) P = cmulz(P, mk<double>(ek.x / a, ek.y / a));
    }
  }
  // pads: decoupled, distinct and above every eigenvalue (Gershgorin)
  const double big = 2.0 * (dmax + 2.0 * bmax) + 1.0;
  for (int k = n; k < N; ++k) Rd[k] = big * (1.0 + (double)(k - n + 1) / (double)N);
  for (int k = n - 1; k < N - 1; ++k) Rb[k] = 0.0;
}

// leaf matrices (dense complex mL x mL, consecutive) with the tearing corrections
__global__ void k_dc_leaves(int N, int L, int mL, const double* __restrict__ Rd, const double* __restrict__ Rb,
                            z64* Al) {
  const int64_t tot = (int64_t)L * mL * mL;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot; x += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(x / ((int64_t)mL * mL));
    const int rem = (int)(x % ((int64_t)mL * mL));
    const int r = rem % mL, c = rem / mL;
    const int s = i * mL;
    double v = 0.0;
    if (r == c) {
      v = Rd[s + r];
      if (r == 0 && i > 0) v -= Rb[s - 1];
      if (r == mL - 1 && i < L - 1) v -= Rb[s + mL - 1];
    } else if (r == c + 1 || c == r + 1) {
      v = Rb[s + min(r, c)];
    }
    Al[x] = mk<double>(v, 0.0);
  }
}

// block-diagonal eigenvector matrix of the leaves into Qa (N x N); Qb zeroed
__global__ void k_dc_init(int N, int mL, const double* __restrict__ wl, const z64* __restrict__ Vl, double* Qa,
                          double* Qb, double* D) {
  const int64_t tot = (int64_t)N * N;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot; x += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(x % N), c = (int)(x / N);
    const int i = r / mL;
    double v = 0.0;
    if (c / mL == i) v = Vl[(int64_t)i * mL * mL + (r - i * mL) + (int64_t)(c - i * mL) * mL].x;
    Qa[x] = v;
    Qb[x] = 0.0;
    if (r == 0) D[c] = wl[c];
  }
}

// merge step A (one work-group per merge of two blocks of size sz): the
// sorted poles and the rank-one vector z, deflation (one thread), the
// deflation rotations on the block's columns, the non-deflated poles
__global__ void __launch_bounds__(1024) k_dc_merge_a(DcBig S, int sz, double* Q) {
  const int N = S.N, m = 2 * sz, j = blockIdx.x, s = j * m, n1 = sz, n2 = sz, t = threadIdx.x;
  const double rho = 2.0 * S.Rb[s + n1 - 1];
  for (int g = t; g < m; g += blockDim.x) {
    const int jj = g;
    const double x = S.D[s + g];
    int lo = 0, cnt;
    if (jj < n1) {  // entries of the right half strictly below x
      cnt = n2;
      while (cnt > 0) {
        const int h = cnt >> 1;
        if (S.D[s + n1 + lo + h] < x) {
          lo += h + 1;
          cnt -= h + 1;
        } else {
          cnt = h;
        }
      }
    } else {  // entries of the left half at or below x
      cnt = n1;
      while (cnt > 0) {
        const int h = cnt >> 1;
        if (S.D[s + lo + h] <= x) {
          lo += h + 1;
          cnt -= h + 1;
        } else {
          cnt = h;
        }
      }
    }
    const int q = (jj < n1 ? jj : jj - n1) + lo;
    S.srt[s + q] = jj;
    S.dl[s + q] = x;
    const int64_t col = (int64_t)(s + jj) * N;
    S.zz[s + q] = (jj < n1 ? Q[(s + n1 - 1) + col] : Q[(s + n1) + col]) * 0.7071067811865476;
  }
  __syncthreads();
  if (t == 0) {
    double dmax = 0.0, zmax = 0.0;
    for (int q = 0; q < m; ++q) {
      dmax = fmax(dmax, fabs(S.dl[s + q]));
      zmax = fmax(zmax, fabs(S.zz[s + q]));
    }
    const double tol = 8.0 * kEps * fmax(dmax, rho * zmax);
    int K = 0, nd = 0, nr = 0, pj = -1;
    for (int jj = 0; jj < m; ++jj) {
      if (rho * fabs(S.zz[s + jj]) <= tol) {
        S.dfl[s + nd++] = jj;
        continue;
      }
      if (pj < 0) {
        pj = jj;
        continue;
      }
      const double zs = S.zz[s + pj], zc = S.zz[s + jj];
      const double tau = hypot(zc, zs);
      const double c = zc / tau, sn = -zs / tau;
      const double tt = S.dl[s + jj] - S.dl[s + pj];
      if (fabs(tt * c * sn) <= tol) {
        S.zz[s + jj] = tau;
        S.zz[s + pj] = 0.0;
        S.ra[s + nr] = S.srt[s + pj];
        S.rb[s + nr] = S.srt[s + jj];
        S.rc[s + nr] = c;
        S.rs[s + nr] = sn;
        ++nr;
        const double dp = S.dl[s + pj], dj = S.dl[s + jj];
        S.dl[s + pj] = c * c * dp + sn * sn * dj;
        S.dl[s + jj] = sn * sn * dp + c * c * dj;
        S.dfl[s + nd++] = pj;
        pj = jj;
      } else {
        S.nd[s + K++] = pj;
        pj = jj;
      }
    }
    if (pj >= 0) S.nd[s + K++] = pj;
    S.Km[j] = K;
    S.nrot[j] = nr;
    S.ndf[j] = nd;
  }
  __syncthreads();
  const int nr = S.nrot[j], K = S.Km[j];
  for (int R = t; R < m; R += blockDim.x) {
    for (int q = 0; q < nr; ++q) {
      const int64_t ca = (int64_t)(s + S.ra[s + q]) * N, cb = (int64_t)(s + S.rb[s + q]) * N;
      const double c = S.rc[s + q], sn = S.rs[s + q];
      const double qa = Q[s + R + ca], qb = Q[s + R + cb];
      Q[s + R + ca] = c * qa + sn * qb;
      Q[s + R + cb] = -sn * qa + c * qb;
    }
  }
  for (int i = t; i < K; i += blockDim.x) {
    S.tv[s + i] = S.dl[s + S.nd[s + i]];
    S.nrm[s + i] = S.zz[s + S.nd[s + i]];
  }
}

// secular roots, 8 lanes per root, 128 roots per work-group
__global__ void __launch_bounds__(1024) k_dc_secular(DcBig S, int sz, int chunks) {
  const int m = 2 * sz, j = blockIdx.x / chunks, s = j * m;
  const int i = (blockIdx.x % chunks) * 128 + (threadIdx.x >> 3), lane8 = threadIdx.x & 7;
  const int K = S.Km[j];
  if (i >= K) return;
  const double rho = 2.0 * S.Rb[s + sz - 1];
  int o;
  const double tau = secular_root(S.tv + s, S.nrm + s, K, rho, i, lane8, o);
  if (lane8 == 0) {
    S.org[s + i] = o;
    S.tau[s + i] = tau;
  }
}

// merge step B (one work-group per merge): Loewner weights, column norms of U,
// output order; then U (K x K, scaled columns) and the gathered source columns
// Qg (m x K) for the product
__global__ void __launch_bounds__(1024) k_dc_merge_b(DcBig S, int sz, const double* Q, double* Ub, double* Qgb) {
  const int N = S.N, m = 2 * sz, j = blockIdx.x, s = j * m, t = threadIdx.x;
  const int K = S.Km[j], nd = S.ndf[j];
  const double* dK = S.tv + s;
  for (int i = t; i < K; i += blockDim.x) {
    const double di = dK[i];
    double wv = (di - dK[S.org[s + i]]) - S.tau[s + i];
    for (int k = 0; k < K; ++k)
      if (k != i) wv *= ((di - dK[S.org[s + k]]) - S.tau[s + k]) / (di - dK[k]);
    S.zh[s + i] = copysign(sqrt(fmax(-wv, 0.0)), S.nrm[s + i]);
    S.src[s + i] = s + S.srt[s + S.nd[s + i]];
  }
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += 128) {
    const int k = k0 + (t >> 3), lane8 = t & 7;
    double acc = 0.0;
    if (k < K) {
      const double lo = dK[S.org[s + k]], tk = S.tau[s + k];
      for (int i = lane8; i < K; i += 8) {
        const double u = S.zh[s + i] / ((dK[i] - lo) - tk);
        acc += u * u;
      }
    }
    acc += dpp_f64<0xB1>(acc);
    acc += dpp_f64<0x4E>(acc);
    acc += dpp_f64<0x141>(acc);
    if (k < K && lane8 == 0) S.cn[s + k] = 1.0 / sqrt(acc);
  }
  if (t == 0) {
    // insertion sort of the deflated values (ascending, stable)
    for (int a2 = 1; a2 < nd; ++a2) {
      const int v = S.dfl[s + a2];
      const double key = S.dl[s + v];
      int b2 = a2 - 1;
      while (b2 >= 0 && S.dl[s + S.dfl[s + b2]] > key) {
        S.dfl[s + b2 + 1] = S.dfl[s + b2];
        --b2;
      }
      S.dfl[s + b2 + 1] = v;
    }
    // outk[q] >= 0: root outk[q]; otherwise the column -outk[q] - 1 (deflated)
    int ia = 0, ib = 0;
    for (int q = 0; q < m; ++q) {
      const double lr = ia < K ? dK[S.org[s + ia]] + S.tau[s + ia] : 0.0;
      const double ld = ib < nd ? S.dl[s + S.dfl[s + ib]] : 0.0;
      if (ib >= nd || (ia < K && lr <= ld)) {
        S.outk[s + q] = ia;
        S.D[s + q] = lr;
        ++ia;
      } else {
        S.outk[s + q] = -(s + S.srt[s + S.dfl[s + ib]] + 1);
        S.D[s + q] = ld;
        ++ib;
      }
    }
  }
  __syncthreads();
  double* U = Ub + (int64_t)j * m * m;
  double* Qg = Qgb + (int64_t)j * m * m;
  for (int64_t x = t; x < (int64_t)K * K; x += blockDim.x) {
    const int i = (int)(x % K), k = (int)(x / K);
    U[x] = S.zh[s + i] / ((dK[i] - dK[S.org[s + k]]) - S.tau[s + k]) * S.cn[s + k];
  }
  for (int64_t x = t; x < (int64_t)m * K; x += blockDim.x) {
    const int r = (int)(x % m), i = (int)(x / m);
    Qg[x] = Q[(s + r) + (int64_t)S.src[s + i] * N];
  }
}

// C (m x K, ld m) = A (m x K, ld m) B (K x K, ld K) for every merge (blockIdx.z),
// K = Km[merge]; 64 x 64 tiles, 256 threads with 4 x 4 results each
__global__ void __launch_bounds__(256) k_dc_gemm(int m, const int* __restrict__ Km, const double* __restrict__ Ab,
                                                 const double* __restrict__ Bb, double* Cb) {
  const int j = blockIdx.z;
  const int K = Km[j];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (c0 >= K || r0 >= m) return;
  const int64_t stride = (int64_t)m * m;
  const double* A = Ab + j * stride;
  const double* B = Bb + j * stride;
  double* C = Cb + j * stride;
  __shared__ double As[16][65], Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int rr = e & 63, kk = e >> 6, r = r0 + rr, k = k0 + kk;
      As[kk][rr] = (r < m && k < K) ? A[r + (int64_t)k * m] : 0.0;
    }
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int kk = e & 15, cc = e >> 4, k = k0 + kk, c = c0 + cc;
      Bs[kk][cc] = (k < K && c < K) ? B[k + (int64_t)c * K] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][tx + 16 * u];
        b[u] = Bs[kk][ty + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + tx + 16 * u, c = c0 + ty + 16 * v;
      if (r < m && c < K) C[r + (int64_t)c * m] = acc[u][v];
    }
}

// merged block columns into the other buffer: roots from the product, the
// deflated columns moved; grid (m columns, merges)
__global__ void __launch_bounds__(256) k_dc_scatter(DcBig S, int sz, const double* Qold, const double* Qob,
                                                    double* Qnew) {
  const int N = S.N, m = 2 * sz, j = blockIdx.y, s = j * m, q = blockIdx.x;
  const int o = S.outk[s + q];
  double* dst = Qnew + (int64_t)(s + q) * N + s;
  if (o >= 0) {
    const double* src = Qob + (int64_t)j * m * m + (int64_t)o * m;
    for (int r = threadIdx.x; r < m; r += blockDim.x) dst[r] = src[r];
  } else {
    const double* src = Qold + (int64_t)(-o - 1) * N + s;
    for (int r = threadIdx.x; r < m; r += blockDim.x) dst[r] = src[r];
  }
}

// V = P Z (n x n leading part), w = eigenvalues
__global__ void k_dc_output(int n, int N, const double* __restrict__ Q, const double* __restrict__ D,
                            const z64* __restrict__ Ph, z64* V, int64_t ldv, double* w) {
  const int64_t tot = (int64_t)n * n;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < tot; x += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(x % n), c = (int)(x / n);
    const z64 P = Ph[r];
    const double z = Q[r + (int64_t)c * N];
    V[r + (int64_t)c * ldv] = mk<double>(P.x * z, P.y * z);
    if (r == 0) w[c] = D[c];
  }
}

template <typename T> T* carve(char*& p, size_t count) {
  T* r = reinterpret_cast<T*>(p);
  p += (sizeof(T) * count + 255) / 256 * 256;
  return r;
}

}  // namespace

bool heev_big(hipStream_t st, int n, const z64* A, int64_t lda, int64_t sA, double* w, int64_t sw, z64* V,
              int64_t ldv, int64_t sV, int batch, DevMem& scr) {
  if (n <= kDcMax || n > kDcBig) return false;
  int L = 1;
  while ((n + L - 1) / L > kDcMax) L *= 2;
  const int mL = (n + L - 1) / L, N = L * mL;
  // scratch: the Householder stage, the leaves, two N x N eigenvector
  // buffers, the per-merge U, Qg and the product (N^2 each), the per-index
  // arrays; laid out once from offset 0 to size it
  const size_t nn = (size_t)n * n, NN = (size_t)N * N;
  const int64_t per = (int64_t)((heev_dc_scratch(mL) + 255) / 256 * 256 / sizeof(double));
  z64 *Ah, *Vh, *e, *Ph, *Al, *Vl;
  double *dd, *bt, *wl, *lscr, *Qa, *Qb, *Ub, *Qg, *Qo;
  char* tscr;
  DcBig S;
  auto layout = [&](char* p) {
    Ah = carve<z64>(p, nn);
    Vh = carve<z64>(p, nn);
    e = carve<z64>(p, n);
    Ph = carve<z64>(p, n);
    dd = carve<double>(p, n);
    bt = carve<double>(p, n);
    tscr = carve<char>(p, tridiag_scratch(n));
    Al = carve<z64>(p, (size_t)L * mL * mL);
    Vl = carve<z64>(p, (size_t)L * mL * mL);
    wl = carve<double>(p, (size_t)L * mL);
    lscr = carve<double>(p, (size_t)per * L);
    Qa = carve<double>(p, NN);
    Qb = carve<double>(p, NN);
    Ub = carve<double>(p, NN);
    Qg = carve<double>(p, NN);
    Qo = carve<double>(p, NN);
    S.n = n;
    S.N = N;
    S.L = L;
    S.mL = mL;
    S.Rd = carve<double>(p, N);
    S.Rb = carve<double>(p, N);
    S.D = carve<double>(p, N);
    S.dl = carve<double>(p, N);
    S.zz = carve<double>(p, N);
    S.tv = carve<double>(p, N);
    S.nrm = carve<double>(p, N);
    S.zh = carve<double>(p, N);
    S.cn = carve<double>(p, N);
    S.rc = carve<double>(p, N);
    S.rs = carve<double>(p, N);
    S.tau = carve<double>(p, N);
    S.srt = carve<int>(p, N);
    S.nd = carve<int>(p, N);
    S.dfl = carve<int>(p, N);
    S.ra = carve<int>(p, N);
    S.rb = carve<int>(p, N);
    S.org = carve<int>(p, N);
    S.outk = carve<int>(p, N);
    S.src = carve<int>(p, N);
    S.Km = carve<int>(p, L);
    S.nrot = carve<int>(p, L);
    S.ndf = carve<int>(p, L);
    return p;
  };
  // sized by a layout from the (aligned) address 256, not from null
  const size_t need = (size_t)(reinterpret_cast<uintptr_t>(layout(reinterpret_cast<char*>((uintptr_t)256))) - 256) + 256;
  scr.ensure(need);
  layout(static_cast<char*>(scr.p));
  for (int b = 0; b < batch; ++b) {
    // 1. Householder reduction of the Hermitian part of A
    HIPCK(hipMemcpy2DAsync(Ah, sizeof(z64) * n, A + b * sA, sizeof(z64) * lda, sizeof(z64) * n, n,
                           hipMemcpyDeviceToDevice, st));
    hermitize(st, n, Ah, n, 0, 1);
    tridiag_reduce(st, n, Ah, n, dd, e, Vh, bt, tscr);
    // 2.-3. real tridiagonal, pads, leaves
    hipLaunchKernelGGL(k_dc_phase, dim3(1), dim3(64), 0, st, n, N, dd, e, Ph, S.Rd, S.Rb);
    const int64_t lt = (int64_t)L * mL * mL;
    hipLaunchKernelGGL(k_dc_leaves, dim3((unsigned)std::min<int64_t>(1024, (lt + 255) / 256)), dim3(256), 0, st, N, L,
                       mL, S.Rd, S.Rb, Al);
    heev_dc_raw(st, mL, Al, mL, (int64_t)mL * mL, wl, mL, Vl, mL, (int64_t)mL * mL, L, lscr);
    hipLaunchKernelGGL(k_dc_init, dim3((unsigned)std::min<int64_t>(4096, ((int64_t)NN + 255) / 256)), dim3(256), 0,
                       st, N, mL, wl, Vl, Qa, Qb, S.D);
    HIPCK(hipGetLastError());
    // 4. merges
    double* Qcur = Qa;
    double* Qnxt = Qb;
    for (int sz = mL; sz < N; sz *= 2) {
      const int m = 2 * sz, nm = N / m, chunks = (m + 127) / 128;
      hipLaunchKernelGGL(k_dc_merge_a, dim3(nm), dim3(1024), 0, st, S, sz, Qcur);
      hipLaunchKernelGGL(k_dc_secular, dim3(nm * chunks), dim3(1024), 0, st, S, sz, chunks);
      hipLaunchKernelGGL(k_dc_merge_b, dim3(nm), dim3(1024), 0, st, S, sz, Qcur, Ub, Qg);
      hipLaunchKernelGGL(k_dc_gemm, dim3((m + 63) / 64, (m + 63) / 64, nm), dim3(256), 0, st, m, S.Km, Qg, Ub, Qo);
      hipLaunchKernelGGL(k_dc_scatter, dim3(m, nm), dim3(256), 0, st, S, sz, Qcur, Qo, Qnxt);
      HIPCK(hipGetLastError());
      std::swap(Qcur, Qnxt);
    }
    // 5. back to the basis of A
    z64* Vb = V + b * sV;
    hipLaunchKernelGGL(k_dc_output, dim3((unsigned)std::min<int64_t>(4096, ((int64_t)nn + 255) / 256)), dim3(256), 0,
                       st, n, N, Qcur, S.D, Ph, Vb, ldv, w + b * sw);
    apply_refl(st, n, n, Vh, bt, Vb, ldv, 0);
    HIPCK(hipGetLastError());
  }
  return true;
}

}  // namespace eahp
