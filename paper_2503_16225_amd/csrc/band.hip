// Projected Sylvester solve of the block FOM (Algorithm 4) for large projected
// systems: (A - s_l I) y_l = c_l for every column l of the right-hand side,
// A (q x q) Hermitian, q > 512.
//
// A is reduced to Hermitian band form B = Q^H A Q of bandwidth kBw by blocked
// Householder transformations (the first stage of a two-stage
// tridiagonalisation).  For every panel of kBw columns:
//   * the block below the band, P (m x kBw), is factored P = H [R; 0] with
//     H = H_0 ... H_{kBw-1}, H_i = I - beta_i v_i v_i^H (a cooperative kernel:
//     one exchange of partial sums between the work-groups per column);
//   * the trailing matrix A22 (m x m) becomes H^H A22 H through the compact
//     WY form H = I - V T V^H, as complex products on the matrix cores:
//       X = A22 V,  Y = X T,  Z = Y - 1/2 V (T^H V^H Y),
//       A22 <- A22 - V Z^H - Z V^H.
// Every shifted system is then a banded solve with partial pivoting, one
// work-group per shift, its active rows in registers:
//   y_l = Q (B - s_l I)^-1 Q^H c_l,
// with Q^H and Q applied as blocked reflector products.  The result is the
// Galerkin solution of the projected equation, the same as through a
// tridiagonal reduction or an eigendecomposition of A (it is unique); the
// O(q^3) part of the work runs as matrix products instead of a matrix-vector
// product with the whole trailing matrix per column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "devcommon.h"
#include "exchange.h"
#include "kernels.h"
#include "ops.h"

namespace eahp {

namespace {
constexpr int kBw = 64;             // bandwidth = panel width (one column per lane)
constexpr int kRw = 2 * kBw + 1;    // stored entries per row of B
constexpr int kWs = kBw + 1;        // active rows of the banded elimination
constexpr int kPanelRpt = 8;        // panel rows per thread (128 rows per work-group)
constexpr int kPanelRows = 16 * kPanelRpt;
constexpr size_t kUbufMax = size_t(8) << 30;  // bytes of eliminated rows held at once
}  // namespace

__global__ void k_band_fill(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Householder QR of the panel P (m x kBw, ld ldp) below the band.  Work-group
// g holds rows g * kPanelRows .. in registers: lane j of wave w has column j
// of rows g * kPanelRows + w + 16 s.  Step i (column i, rows i..m-1):
//   D_j = x^H p_j over rows >= i, x = column i (one exchange of per-group
//   partial sums, added in a fixed order: every work-group gets the same
//   values), r_j = p_{i,j} (row i, held by work-group 0);
//   alpha = -(x_i/|x_i|) ||x||, v = x - alpha e_i, beta = 2 / v^H v,
//   w_j = beta v^H p_j = beta (D_j - conj(alpha) r_j), p_j -= v w_j.
// Outputs: R (upper triangle) over the first rows of P, v_i (zero above row
// i, v_i[i] = x_i - alpha) into columns 0..kBw-1 and 2kBw..3kBw-1 of V3 and
// into Vh, beta_i.  A timed-out exchange sets err.
template <int RPT>
__global__ void __launch_bounds__(1024) k_band_panel(int m, z64* P, int64_t ldp, z64* V3, int64_t ldv3, z64* Vh,
                                                     int64_t ldvh, double* beta, z64* part, z64* rowv, int* err) {
  __shared__ z64 red[16][64];
  __shared__ z64 red2[16][64];
  __shared__ z64 rsh[64];
  __shared__ z64 v0s[64];
  __shared__ double bsh[64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const int rbase = g * 16 * RPT + w;
  z64 a[RPT];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = rbase + 16 * s;
    a[s] = r < m ? P[r + (int64_t)lane * ldp] : mk<double>(0.0, 0.0);
  }
  bool ok = true;
  const int ns = min(kBw, m);
  for (int i = 0; i < ns; ++i) {
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = rbase + 16 * s;
      double xr = readlane_f64(a[s].x, i), xi = readlane_f64(a[s].y, i);
      if (r < i) xr = xi = 0.0;
      ax += xr * a[s].x + xi * a[s].y;  // conj(x) p
      ay += xr * a[s].y - xi * a[s].x;
    }
    red[w][lane] = mk<double>(ax, ay);
    __syncthreads();
    if (w == 0) {
      z64 t = red[0][lane];
      for (int ww = 1; ww < 16; ++ww) t = cadd<double>(t, red[ww][lane]);
      xch::put_z(part + ((int64_t)i * G + g) * 64 + lane, t);
    }
    if (g == 0 && w == (i & 15)) {  // row i: work-group 0, wave i % 16, slot i / 16
#pragma unroll
      for (int s = 0; s < 4 && s < RPT; ++s)
        if (s == (i >> 4)) xch::put_z(rowv + (int64_t)i * 64 + lane, a[s]);
    }
    // wave w adds the partials of work-groups w, w + 16, ... in order
    z64 pp = mk<double>(0.0, 0.0);
    for (int gg = w; gg < G; gg += 16) pp = cadd<double>(pp, xch::poll_z(part + ((int64_t)i * G + gg) * 64 + lane, ok));
    red2[w][lane] = pp;
    if (w == 15) rsh[lane] = xch::poll_z(rowv + (int64_t)i * 64 + lane, ok);
    __syncthreads();
    z64 D = red2[0][lane];
    for (int ww = 1; ww < 16; ++ww) D = cadd<double>(D, red2[ww][lane]);
    const z64 rj = rsh[lane];
    const double xn2 = fmax(readlane_f64(D.x, i), 0.0);
    const z64 x0 = rsh[i];
    const double xn = sqrt(xn2);
    const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
    const z64 alpha = a0 > 0 ? mk<double>(-x0.x / a0 * xn, -x0.y / a0 * xn) : mk<double>(-xn, 0.0);
    const z64 v0 = csub<double>(x0, alpha);
    const double vv = (xn2 - a0 * a0) + (v0.x * v0.x + v0.y * v0.y);
    const double b = vv > 0 ? 2.0 / vv : 0.0;
    const z64 ca = cjmul<double>(alpha, rj);  // conj(alpha) r_j
    const z64 wj = mk<double>(b * (D.x - ca.x), b * (D.y - ca.y));
    if (lane > i) {
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = rbase + 16 * s;
        const z64 xv = mk<double>(readlane_f64(a[s].x, i), readlane_f64(a[s].y, i));
        if (r > i) a[s] = csub<double>(a[s], cmul<double>(xv, wj));
        else if (r == i) a[s] = csub<double>(a[s], cmul<double>(v0, wj));
      }
    } else if (lane == i) {
#pragma unroll
      for (int s = 0; s < RPT; ++s)
        if (rbase + 16 * s == i) a[s] = alpha;
    }
    if (threadIdx.x == 0) {
      v0s[i] = v0;
      bsh[i] = b;
    }
  }
  __syncthreads();
  if (!ok) err[0] = 1;
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int r = rbase + 16 * s, j = lane;
    if (r >= m) continue;
    if (r <= j) P[r + (int64_t)j * ldp] = a[s];
    const z64 vj = (j >= ns || r < j) ? mk<double>(0.0, 0.0) : (r == j ? v0s[j] : a[s]);
    V3[r + (int64_t)j * ldv3] = vj;
    V3[r + (int64_t)(2 * kBw + j) * ldv3] = vj;
    Vh[r + (int64_t)j * ldvh] = vj;
  }
  if (g == 0 && threadIdx.x < kBw) beta[threadIdx.x] = (int)threadIdx.x < ns ? bsh[threadIdx.x] : 0.0;
}

// Compact WY factor of H = H_0 ... H_{nb-1} = I - V T V^H from G = V^H V
// (nb x nb, ld nb) and beta: T^-1 = diag(1/beta) + (strictly upper part of G),
// so column j of T is T_jj = beta_j, T_ij = -beta_i sum_{k=i+1..j} G_ik T_kj
// (i < j), by back substitution; one thread per column.
__global__ void __launch_bounds__(64) k_band_form_t(const z64* __restrict__ G, const double* __restrict__ beta,
                                                    z64* __restrict__ T) {
  __shared__ z64 Gs[kBw * kBw];
  __shared__ z64 Ts[kBw * kBw];
  const int j = threadIdx.x;
  for (int e = j; e < kBw * kBw; e += 64) {
    Gs[e] = G[e];
    Ts[e] = mk<double>(0.0, 0.0);
  }
  __syncthreads();
  Ts[j + kBw * j] = mk<double>(beta[j], 0.0);
  for (int i = j - 1; i >= 0; --i) {
    double sx = 0.0, sy = 0.0;
    for (int k = i + 1; k <= j; ++k) {
      const z64 gk = Gs[i + kBw * k], tk = Ts[k + kBw * j];
      sx += gk.x * tk.x - gk.y * tk.y;
      sy += gk.x * tk.y + gk.y * tk.x;
    }
    Ts[i + kBw * j] = mk<double>(-beta[i] * sx, -beta[i] * sy);
  }
  __syncthreads();
  for (int e = j; e < kBw * kBw; e += 64) T[e] = Ts[e];
}

// Rows of the band matrix: RB[r * kRw + t] = B[r][r - kBw + t] (t = 0..2kBw),
// zero outside the matrix; entries on and below the diagonal come from the
// lower triangle of A, the others as conjugates of their mirror.
__global__ void k_band_rows(int q, const z64* __restrict__ A, int64_t lda, z64* __restrict__ RB) {
  const int64_t n = (int64_t)q * kRw;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / kRw), t = (int)(e - (int64_t)r * kRw);
    const int c = r - kBw + t;
    z64 v = mk<double>(0.0, 0.0);
    if (c >= 0 && c < q) {
      if (c <= r) v = A[r + (int64_t)c * lda];
      else {
        const z64 u = A[c + (int64_t)r * lda];
        v = mk<double>(u.x, -u.y);
      }
    }
    RB[e] = v;
  }
}

// Banded solve with partial pivoting, (B - s I) y = c, one shift per
// work-group (shift l0 + blockIdx.x, right-hand side and solution in column
// l0 + blockIdx.x of Y).
//
// Elimination step k picks the pivot among the kBw + 1 rows not yet
// eliminated (all of column k's non-zeros lie in them); the pivot row has
// its non-zeros in columns k .. k + 2kBw.  The active rows are held in
// registers over columns k+1 .. k+2kBw: thread t keeps column slot t % 128
// (column c in slot c % 128) of the row slots t / 128 + 8 i.  A row keeps its
// slot until it becomes the pivot; the row that enters the window (row
// k + kBw + 1, whose band spans columns k+1 .. k+2kBw+1) takes the freed
// slot.  Column k is kept apart in LDS for the pivot search and the
// multipliers; after the step, column k+1 moves there and its register slot
// takes column k + 2kBw + 1 (zero in every row but the entering one).  A
// step has two barriers: every wave finds the pivot slot itself (the same
// arg-max over the same values) and each thread forms the multipliers of its
// own rows, while the pivot column, the right-hand sides and the row numbers
// of the next step go to the other of two LDS buffers.
// Eliminated rows go to Ubuf (row k: U[k][0] the pivot, U[k][1 + d] the entry
// in column k + 1 + d) and the transformed right-hand side into y; the
// triangular system U y = z is then solved backwards by one wave, its rows
// staged through LDS by the whole work-group.
constexpr int kGeppChunk = 32;  // rows of U per LDS stage in the backward solve
__device__ __forceinline__ z64 zz() { return mk<double>(0.0, 0.0); }

__global__ void __launch_bounds__(1024) k_band_gepp(int q, const z64* __restrict__ RB, const double* __restrict__ shift,
                                                    z64* __restrict__ Y, int64_t ldy, z64* __restrict__ Ubuf, int l0) {
  // column k of the active rows, their right-hand sides and row numbers, by
  // slot; step k reads buffer k & 1 and writes the other
  __shared__ z64 pcb[2][kWs];
  __shared__ z64 rhsb[2][kWs];
  __shared__ int ridb[2][kWs];
  __shared__ z64 urow[2 * kBw];
  __shared__ z64 ent[kRw + 1];  // the entering row (d = 0..2kBw) and its right-hand side
  __shared__ z64 ust[2][kGeppChunk][kRw + 1];  // backward solve: rows of U, then z
  const int l = l0 + blockIdx.x;
  const double sft = shift[l];
  z64* y = Y + (int64_t)l * ldy;
  z64* U = Ubuf + (int64_t)blockIdx.x * q * kRw;
  const int t = threadIdx.x, cs = t & 127, rg = t >> 7, lane = t & 63;
  auto bval = [&](int r, int c) __attribute__((always_inline)) -> z64 {
    if (r >= q || c < 0 || c >= q || c < r - kBw || c > r + kBw) return zz();
    z64 v = RB[(int64_t)r * kRw + (c - r + kBw)];
    if (r == c) v.x -= sft;
    return v;
  };
  // element d = t of the row entering at step kk (d = kRw: its right-hand side)
  auto fetch = [&](int kk) __attribute__((always_inline)) -> z64 {
    const int re = kk + kWs;
    if (re >= q) return zz();
    if (t == kRw) return y[re];
    const int c = kk + 1 + t;
    if (t > kRw || c >= q) return zz();
    z64 v = RB[(int64_t)re * kRw + t];
    if (t == kBw) v.x -= sft;
    return v;
  };
  // the thread's row slots rg + 8 i (i < 8), real and imaginary parts in two
  // 8-wide vector registers (a slot chosen at run time is read by indexed
  // register moves), and slot 64 (row group 0) in a register pair of its own
  d8 wre, wim;
  z64 w64 = zz();
  const int c0 = cs == 0 ? 2 * kBw : cs;  // columns 1 .. 2kBw at step 0
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const z64 v = bval(rg + 8 * i, c0);
    wre[i] = v.x;
    wim[i] = v.y;
  }
  if (rg == 0) w64 = bval(kBw, c0);
  if (t < kWs) {
    pcb[0][t] = bval(t, 0);
    rhsb[0][t] = t < q ? y[t] : zz();
    ridb[0][t] = t < q ? t : -1;
  }
  // one elimination step; e holds the entering row of step k (loaded three
  // steps ahead) and takes that of step k + 3
  auto step = [&](int k, z64& e) __attribute__((always_inline)) {
    const z64* pc = pcb[k & 1];
    const z64* rhs = rhsb[k & 1];
    const int* rid = ridb[k & 1];
    z64* pcn = pcb[(k & 1) ^ 1];
    z64* rhsn = rhsb[(k & 1) ^ 1];
    int* ridn = ridb[(k & 1) ^ 1];
    // (A) the entering row into LDS; the pivot slot, found by every wave
    // alike (the same reduction on the same values); the pivot row
    if (t <= kRw) ent[t] = e;
    e = fetch(k + 3);
    int sp;
    {
      const z64 pv = pc[lane];
      double v = rid[lane] >= 0 ? pv.x * pv.x + pv.y * pv.y : -1.0;
      int ix = lane;
      if (lane == 0) {
        const z64 p64 = pc[kBw];
        argmax_merge(v, ix, rid[kBw] >= 0 ? p64.x * p64.x + p64.y * p64.y : -1.0, kBw);
      }
      wave_argmax(v, ix);
      sp = ix;
    }
    if (sp == kBw ? rg == 0 : rg == (sp & 7)) {
      const z64 v = sp == kBw ? w64 : mk<double>(wre[sp >> 3], wim[sp >> 3]);
      urow[cs] = v;
      U[(int64_t)k * kRw + 1 + ((cs - k - 1) & 127)] = v;
    }
    const z64 pp = pc[sp];
    if (t == 0) {
      U[(int64_t)k * kRw] = pp;
      y[k] = rhs[sp];
    }
    __syncthreads();
    // (B) elimination, each thread forming the multipliers of its rows;
    // column k+1 into the other buffer; the entering row into slot sp
    const double den = pp.x * pp.x + pp.y * pp.y;
    const z64 inv = mk<double>(pp.x / den, -pp.y / den);
    const int csn = (k + 1) & 127;
    const z64 u = urow[cs];
    const int dd = (cs - k - 1) & 127;
    const z64 ev = ent[dd == 0 ? 2 * kBw : dd];
    auto update = [&](int rs, z64 w) __attribute__((always_inline)) -> z64 {
      z64 val;
      if (rs == sp) {
        val = ev;
        if (cs == csn) pcn[rs] = ent[0];
      } else {
        const z64 lr = cmul<double>(pc[rs], inv);
        val = csub<double>(w, cmul<double>(lr, u));
        if (cs == csn) {
          pcn[rs] = val;
          val = zz();
        }
      }
      return val;
    };
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const z64 val = update(rg + 8 * i, mk<double>(wre[i], wim[i]));
      wre[i] = val.x;
      wim[i] = val.y;
    }
    if (rg == 0) w64 = update(kBw, w64);
    if (t < kWs) {
      if (t == sp) {
        const int re = k + kWs;
        rhsn[t] = ent[kRw];
        ridn[t] = re < q ? re : -1;
      } else {
        const z64 lt = cmul<double>(pc[t], inv);
        rhsn[t] = csub<double>(rhs[t], cmul<double>(lt, rhs[sp]));
        ridn[t] = rid[t];
      }
    }
    __syncthreads();
  };
  z64 e0 = fetch(0), e1 = fetch(1), e2 = fetch(2);
  __syncthreads();
  for (int k = 0; k < q; k += 3) {
    step(k, e0);
    if (k + 1 < q) step(k + 1, e1);
    if (k + 2 < q) step(k + 2, e2);
  }
  // ---- backward solve U y = z.  Chunks of kGeppChunk rows, from the last:
  // every thread loads its share of the next chunk while wave 0 solves the
  // current one from LDS.  Lane j of wave 0 holds y[k+1+j] and y[k+65+j].
  const int nch = (q + kGeppChunk - 1) / kGeppChunk;
  constexpr int kPer = kGeppChunk * (kRw + 1);
  auto stage_ld = [&](int ch, z64* vals) __attribute__((always_inline)) {
    const int r0 = ch * kGeppChunk;
    for (int e = t, u = 0; u < (kPer + 1023) / 1024; e += 1024, ++u) {
      z64 v = zz();
      if (e < kPer) {
        const int rr = e / (kRw + 1), cc = e - rr * (kRw + 1);
        const int k = r0 + rr;
        if (k < q) v = cc < kRw ? U[(int64_t)k * kRw + cc] : y[k];
      }
      vals[u] = v;
    }
  };
  auto stage_st = [&](int buf, const z64* vals) __attribute__((always_inline)) {
    for (int e = t, u = 0; u < (kPer + 1023) / 1024; e += 1024, ++u)
      if (e < kPer) (&ust[buf][0][0])[e] = vals[u];
  };
  z64 sv[(kPer + 1023) / 1024];
  stage_ld(nch - 1, sv);
  stage_st((nch - 1) & 1, sv);
  __syncthreads();
  z64 ya = zz(), yb = zz();
  for (int ch = nch - 1; ch >= 0; --ch) {
    if (ch > 0) stage_ld(ch - 1, sv);
    if (t < 64) {
      const int r0 = ch * kGeppChunk;
      const int rr_hi = min(kGeppChunk, q - r0) - 1;
      for (int rr = rr_hi; rr >= 0; --rr) {
        const z64* Ur = ust[ch & 1][rr];
        const z64 ua = Ur[1 + t], ub = Ur[1 + kBw + t], u0 = Ur[0], zk = Ur[kRw];
        double sx = ua.x * ya.x - ua.y * ya.y + ub.x * yb.x - ub.y * yb.y;
        double sy = ua.x * ya.y + ua.y * ya.x + ub.x * yb.y + ub.y * yb.x;
        sx = wave_allsum(sx);
        sy = wave_allsum(sy);
        const double nx = zk.x - sx, ny = zk.y - sy;
        const double den = u0.x * u0.x + u0.y * u0.y;
        const z64 yk = mk<double>((nx * u0.x + ny * u0.y) / den, (ny * u0.x - nx * u0.y) / den);
        if (t == 0) y[r0 + rr] = yk;
        const double a63x = __shfl(ya.x, 63, 64), a63y = __shfl(ya.y, 63, 64);
        const double uax = __shfl_up(ya.x, 1, 64), uay = __shfl_up(ya.y, 1, 64);
        const double ubx = __shfl_up(yb.x, 1, 64), uby = __shfl_up(yb.y, 1, 64);
        ya = t == 0 ? yk : mk<double>(uax, uay);
        yb = t == 0 ? mk<double>(a63x, a63y) : mk<double>(ubx, uby);
      }
    }
    if (ch > 0) stage_st((ch - 1) & 1, sv);
    __syncthreads();
  }
}

// The projected solve for q > kBw (the FOM calls it beyond q = 512): A (q x q,
// ld lda, Hermitian up to rounding; destroyed), s (p shifts), Yt (q x p, ld q:
// the right-hand sides, overwritten by the solutions).
void sylvester_band(hipStream_t st, int q, int p, z64* A, int64_t lda, const double* s, z64* Yt, DevMem& ws,
                    DevMem& part) {
  if (q <= kBw) fail(EAHP_EINVAL, "band reduction: q must exceed the bandwidth");
  if (p <= 0) return;
  const int b = kBw;
  int dev = 0, ncu = 0;
  HIPCK(hipGetDevice(&dev));
  HIPCK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int gmax = (q - b + kPanelRows - 1) / kPanelRows;
  if (gmax > ncu) fail(EAHP_EINVAL, "band reduction: projected system too large for one cooperative panel");
  // shifts per elimination launch: the eliminated rows of each are kept
  const size_t ubytes_shift = sizeof(z64) * (size_t)q * kRw;
  const int nsh = (int)std::max<size_t>(1, std::min<size_t>((size_t)p, kUbufMax / ubytes_shift));
  // workspace: Vh (q x q), beta (q), V3 (q x 3b), X (q x b), G, T, N, M (b x b),
  // RB (q x kRw), exchange slots, error flag, blocked-product scratch, U rows
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t oVh = 0;
  const size_t oBt = oVh + al(sizeof(z64) * (size_t)q * q);
  const size_t oV3 = oBt + al(sizeof(double) * q);
  const size_t oX = oV3 + al(sizeof(z64) * (size_t)q * 3 * b);
  const size_t oSm = oX + al(sizeof(z64) * (size_t)q * b);
  const size_t oRB = oSm + al(sizeof(z64) * 4 * b * b);
  const size_t oSl = oRB + al(sizeof(z64) * (size_t)q * kRw);
  const size_t nslot = (size_t)b * (gmax + 1) * 64;
  const size_t oErr = oSl + al(sizeof(z64) * nslot);
  const size_t oWy = oErr + 256;
  const size_t oU = oWy + al(refl_blocked_scratch(q - b, p));
  ws.ensure(oU + ubytes_shift * nsh);
  char* base = static_cast<char*>(ws.p);
  z64* Vh = reinterpret_cast<z64*>(base + oVh);
  double* bt = reinterpret_cast<double*>(base + oBt);
  z64* V3 = reinterpret_cast<z64*>(base + oV3);
  z64* X = reinterpret_cast<z64*>(base + oX);
  z64* Gm = reinterpret_cast<z64*>(base + oSm);
  z64* Tm = Gm + b * b;
  z64* Nm = Tm + b * b;
  z64* Mm = Nm + b * b;
  z64* RB = reinterpret_cast<z64*>(base + oRB);
  z64* slots = reinterpret_cast<z64*>(base + oSl);
  int* err = reinterpret_cast<int*>(base + oErr);
  void* wy = base + oWy;
  z64* Ubuf = reinterpret_cast<z64*>(base + oU);
  const int64_t ld3 = q;

  hermitize(st, q, A, lda, 0, 1);
  {
    const int64_t nw = (int64_t)2 * q * q;
    hipLaunchKernelGGL(k_band_fill, dim3((unsigned)std::min<int64_t>(4096, (nw + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<unsigned long long*>(Vh), nw, 0ull);
    hipLaunchKernelGGL(k_band_fill, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned long long*>(err), (int64_t)1,
                       0ull);
  }
  {
    // the cooperative panels wait on each other's work-groups: one such grid
    // at a time per process
    std::lock_guard<std::mutex> lk(coop_mutex());
    for (int k0 = 0; k0 + b < q; k0 += b) {
      const int m = q - k0 - b, ns = std::min(b, m);
      const int G = (m + kPanelRows - 1) / kPanelRows;
      z64* P = A + (k0 + b) + (int64_t)k0 * lda;
      z64* part_x = slots;
      z64* rowv = slots + (size_t)ns * G * 64;
      const int64_t nw = (int64_t)2 * ns * (G + 1) * 64;
      hipLaunchKernelGGL(k_band_fill, dim3((unsigned)std::min<int64_t>(1024, (nw + 255) / 256)), dim3(256), 0, st,
                         reinterpret_cast<unsigned long long*>(slots), nw, xch::kEmpty);
      int mm = m;
      int64_t ldp = lda, ldv = ld3, ldh = q;
      z64* Vp = Vh + (int64_t)k0 * q + (k0 + b);
      double* btp = bt + k0;
      void* args[] = {&mm, &P, &ldp, &V3, &ldv, &Vp, &ldh, &btp, &part_x, &rowv, &err};
      HIPCK(hipLaunchCooperativeKernel((const void*)k_band_panel<kPanelRpt>, dim3(G), dim3(1024), args, 0, st));
      // trailing update A22 <- H^H A22 H
      z64* A22 = A + (k0 + b) + (int64_t)(k0 + b) * lda;
      z64* Yb = V3 + (int64_t)b * ld3;
      gemm_hn<double>(st, m, b, b, V3, ld3, V3, ld3, Gm, b, 1.0, 0.0, part);
      hipLaunchKernelGGL(k_band_form_t, dim3(1), dim3(64), 0, st, Gm, bt + k0, Tm);
      gemm_hn<double>(st, m, m, b, A22, lda, V3, ld3, X, ld3, 1.0, 0.0, part);  // A22^H V = A22 V
      gemm_nn<double>(st, m, b, b, X, ld3, Tm, b, 0, Yb, ld3, 1.0, 0.0, 0.0);
      gemm_hn<double>(st, m, b, b, V3, ld3, Yb, ld3, Nm, b, 1.0, 0.0, part);
      gemm_hn<double>(st, b, b, b, Tm, b, Nm, b, Mm, b, 1.0, 0.0, part);
      gemm_nn<double>(st, m, b, b, V3, ld3, Mm, b, 0, Yb, ld3, -0.5, 0.0, 1.0);
      gemm_nn<double>(st, m, 2 * b, m, V3, ld3, Yb, ld3, 1, A22, lda, -1.0, 0.0, 1.0);
    }
    int bad = 0;
    HIPCK(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (bad != 0) fail(EAHP_EDEVICE, "exchange wait of the band reduction timed out");
  }
  hipLaunchKernelGGL(k_band_rows, dim3((unsigned)std::min<int64_t>(8192, ((int64_t)q * kRw + 255) / 256)), dim3(256),
                     0, st, q, A, lda, RB);
  apply_refl_blocked(st, q, b, p, Vh, bt, Yt, q, 1, wy, part);
  for (int l0 = 0; l0 < p; l0 += nsh) {
    const int n = std::min(nsh, p - l0);
    hipLaunchKernelGGL(k_band_gepp, dim3(n), dim3(1024), 0, st, q, RB, s, Yt, (int64_t)q, Ubuf, l0);
  }
  apply_refl_blocked(st, q, b, p, Vh, bt, Yt, q, 0, wy, part);
  HIPCK(hipGetLastError());
}

}  // namespace eahp
