// Register-resident factorisations for the N <= 64 path: one wavefront per matrix, the matrix
// held in VGPRs (one column or one row per lane).
//
// Every step k of a column-pivoted Householder QR or of a Gauss-Jordan inversion works on the
// k-th row (QR) or column (Gauss-Jordan) and everything after it.  Each lane keeps its vector in
// a rotating window: at step k register 0 holds element k, register t holds element k + t; at
// the end of the step the finished element is written out and the window shifts by one with a
// zero (QR) or the step's new column (Gauss-Jordan) entering at the far end.  Register indices
// are therefore the same at every step, the step loop stays rolled (small code, no dynamic
// register indexing, no scratch), and the QR uses windows of 64, 32 and then 16 registers as
// its active part shrinks.  Pivots come from a DPP wave maximum and a ballot; the pivot's
// vector reaches the other lanes through one LDS row (written by the pivot lane, read back as
// broadcasts; LDS operations of one wavefront complete in issue order).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqmc {
namespace stab {

#define DQMC_LDS __attribute__((address_space(3)))
typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double lane_read(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWMASK = 0xf, int BANKMASK = 0xf>
__device__ __forceinline__ double dpp_mov(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, BANKMASK, false);
  int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, BANKMASK, false);
  return __hiloint2double(hi2, lo2);
}

// Maximum over the 64 lanes, returned to all lanes.  Prefix maxima inside each 16-lane row by
// row_shr 1, 2, 4, 8, then row 0 -> row 1 and row 2 -> row 3 (row_bcast:15), then rows 0-1 ->
// rows 2-3 (row_bcast:31): lane 63 holds the maximum.  Lanes whose DPP source is out of range
// or masked keep their own value, which leaves a maximum unchanged.
__device__ __forceinline__ double wave_max64(double x) {
  x = fmax(x, dpp_mov<0x111>(x));
  x = fmax(x, dpp_mov<0x112>(x));
  x = fmax(x, dpp_mov<0x114>(x));
  x = fmax(x, dpp_mov<0x118>(x));
  x = fmax(x, dpp_mov<0x142, 0xa>(x));
  x = fmax(x, dpp_mov<0x143, 0xc>(x));
  return lane_read(x, 63);
}

// Lowest lane whose candidate key equals the wave maximum (keys >= 0; ok = lane is a candidate).
__device__ __forceinline__ int wave_argmax_lane(double key, bool ok, double* kmax) {
  const double mx = wave_max64(ok ? key : -1.0);
  const unsigned long long b = __ballot(ok && key == mx);
  *kmax = mx;
  if (b) return (int)__builtin_ctzll(b);
  const unsigned long long bo = __ballot(ok);   // no key compares equal (NaN): lowest candidate
  return bo ? (int)__builtin_ctzll(bo) : 0;
}

// Orders LDS accesses of this wavefront in the compiler's view (the hardware keeps them in
// issue order).
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

template <int W>
__device__ __forceinline__ void row_store(DQMC_LDS double* dst, const double* v) {
#pragma unroll
  for (int t = 0; t < W; t += 2) *(DQMC_LDS dbl2*)(dst + t) = dbl2{v[t], v[t + 1]};
}

// ------------------------------------------------------------------ column-pivoted Householder QR
// One step j (window width W >= n - j) of the factorisation of the column held by this lane.
// The remaining column of largest norm over rows j.. is the pivot p; its window goes to row j of
// Vb; every other remaining column gets x -= beta (v^T x) v with v = x_p - alpha e_j,
// alpha = -sign(x_pj) |x_p|, beta = 1 / (alpha (alpha - x_pj)).  Row j of the result (R on and
// right of the pivot order's diagonal, Householder vectors below it) is written to X.
template <int NP, int W>
__device__ __forceinline__ void qr_step(int j, double (&x)[NP], double& nrm, bool& used,
                                        int& myrank, int& bad, DQMC_LDS double* X,
                                        DQMC_LDS double* Vb, DQMC_LDS double* vd,
                                        DQMC_LDS double* bt, DQMC_LDS double* dd,
                                        DQMC_LDS double* sgn, DQMC_LDS int* ordv) {
  const int c = threadIdx.x & 63;
  double nx2;
  const int p = wave_argmax_lane(nrm, !used, &nx2);
  DQMC_LDS double* vrow = Vb + j * NP;
  if (c == p) row_store<W>(vrow, x);
  lds_order();
  const double xj = vrow[0];
  const double nx = sqrt(nx2);
  const double alpha = (xj >= 0.0) ? -nx : nx;
  const double beta = (nx > 0.0) ? 1.0 / (alpha * (alpha - xj)) : 0.0;
  const double v0 = xj - alpha;
  if (!(nx > 0.0)) bad = 1;
  if (c == p) { used = true; myrank = j; }
  double w[4] = {v0 * x[0], 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 2; t < W; t += 2) {
    const dbl2 v = *(const DQMC_LDS dbl2*)(vrow + t);
    w[t & 3] += v.x * x[t];
    w[(t + 1) & 3] += v.y * x[t + 1];
  }
  w[1] += vrow[1] * x[1];
  const double ws = used ? 0.0 : ((w[0] + w[1]) + (w[2] + w[3])) * beta;
  const double head = x[0] - ws * v0;
  if (c < NP) X[j * NP + c] = (c == p) ? alpha : head;
  lds_order();
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  {
    const double y = x[1] - ws * vrow[1];
    x[0] = y;
    s[1] = y * y;
  }
#pragma unroll
  for (int t = 2; t < W; t += 2) {
    const dbl2 v = *(const DQMC_LDS dbl2*)(vrow + t);
    const double y0 = x[t] - ws * v.x, y1 = x[t + 1] - ws * v.y;
    x[t - 1] = y0;
    x[t] = y1;
    s[t & 3] += y0 * y0;
    s[(t + 1) & 3] += y1 * y1;
  }
  x[W - 1] = 0.0;
  nrm = (s[0] + s[1]) + (s[2] + s[3]);
  if (c == 0) {
    ordv[j] = p;
    vd[j] = v0;
    bt[j] = beta;
    dd[j] = fabs(alpha);
    sgn[j] = alpha < 0.0 ? -1.0 : 1.0;
  }
}

// Column-pivoted Householder QR of the n x n block of X (LDS, NP x NP, zero padded) by one
// wavefront; lane c holds column c.  Output: X in LAPACK form (R on and above the diagonal of
// the pivot order with R[j][j] = alpha_j at column ordv[j], Householder vectors below);
// Vb row j = the pivot column's window at step j (rows j.. of v_j except v_j[0] = vd[j]);
// bt[j] = beta_j, dd[j] = |alpha_j|, sgn[j] = sign(alpha_j), rank[c] = step of column c.
template <int NP>
__device__ __noinline__ void qr_factor(int n, DQMC_LDS double* X, DQMC_LDS double* Vb,
                                          DQMC_LDS double* vd, DQMC_LDS double* bt,
                                          DQMC_LDS int* rank, DQMC_LDS int* ordv,
                                          DQMC_LDS double* dd, DQMC_LDS double* sgn, int* flags) {
  const int c = threadIdx.x & 63;
  const int cs = c < NP ? c : 0;
  double x[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) x[r] = (c < n) ? X[r * NP + cs] : 0.0;
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < NP; ++r) nrm += x[r] * x[r];
  bool used = (c >= n);
  int myrank = -1, bad = 0;
  int j = 0;
  if constexpr (NP >= 64)
    for (; j < n && n - j > 32; ++j)
      qr_step<NP, 64>(j, x, nrm, used, myrank, bad, X, Vb, vd, bt, dd, sgn, ordv);
  if constexpr (NP >= 32)
    for (; j < n && n - j > 16; ++j)
      qr_step<NP, 32>(j, x, nrm, used, myrank, bad, X, Vb, vd, bt, dd, sgn, ordv);
  for (; j < n; ++j) qr_step<NP, 16>(j, x, nrm, used, myrank, bad, X, Vb, vd, bt, dd, sgn, ordv);
  if (c < NP) rank[c] = (c < n) ? myrank : -1;
  if (bad && c == 0) atomicOr(flags, 8);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// One step j of forming row c of Q = H_0 H_1 ... H_{n-1} (lane c): q <- q - beta (q . v) v on
// columns j.. (window), then column j of the row is final: U[c][j] = Q[c][j] sgn[j].
template <int NP, int W>
__device__ __forceinline__ void qform_step(int j, double (&q)[NP], const DQMC_LDS double* Vb,
                                           const DQMC_LDS double* vd, const DQMC_LDS double* bt,
                                           const DQMC_LDS double* sgn, double* Ud) {
  const int c = threadIdx.x & 63;
  const DQMC_LDS double* vrow = Vb + j * NP;
  const double v0 = vd[j], b = bt[j], sg = sgn[j];
  double w[4] = {v0 * q[0], vrow[1] * q[1], 0.0, 0.0};
#pragma unroll
  for (int t = 2; t < W; t += 2) {
    const dbl2 v = *(const DQMC_LDS dbl2*)(vrow + t);
    w[t & 3] += v.x * q[t];
    w[(t + 1) & 3] += v.y * q[t + 1];
  }
  const double ws = ((w[0] + w[1]) + (w[2] + w[3])) * b;
  if (c < NP) Ud[c * NP + j] = (q[0] - ws * v0) * sg;
  lds_order();
  q[0] = q[1] - ws * vrow[1];
#pragma unroll
  for (int t = 2; t < W; t += 2) {
    const dbl2 v = *(const DQMC_LDS dbl2*)(vrow + t);
    q[t - 1] = q[t] - ws * v.x;
    q[t] = q[t + 1] - ws * v.y;
  }
  q[W - 1] = 0.0;
}

// U = Q Diag(sgn) of the factorisation above, written to Ud (global NP x NP, zero padded).
template <int NP>
__device__ __noinline__ void qr_form_q(int n, const DQMC_LDS double* Vb, const DQMC_LDS double* vd,
                                          const DQMC_LDS double* bt, const DQMC_LDS double* sgn,
                                          double* Ud) {
  const int c = threadIdx.x & 63;
  double q[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) q[t] = (t == c && c < n) ? 1.0 : 0.0;
  int j = 0;
  if constexpr (NP >= 64)
    for (; j < n && n - j > 32; ++j) qform_step<NP, 64>(j, q, Vb, vd, bt, sgn, Ud);
  if constexpr (NP >= 32)
    for (; j < n && n - j > 16; ++j) qform_step<NP, 32>(j, q, Vb, vd, bt, sgn, Ud);
  for (; j < n; ++j) qform_step<NP, 16>(j, q, Vb, vd, bt, sgn, Ud);
  if (c < NP)
    for (; j < NP; ++j) Ud[c * NP + j] = 0.0;
}

// ------------------------------------------------------------------ Gauss-Jordan inversion
// In-place Gauss-Jordan inversion with implicit row pivoting (exchange steps) of
// [[M, 0], [0, I]] (M = the n x n block of an LDS NP x NP matrix) by one wavefront; lane i holds
// row i.  Step k pivots on the remaining row p of largest |A[p][k]| and exchanges the roles of
// x_k and y_p in y = A x:
//   A[p][k] <- 1/a,  A[p][j] <- -A[p][j]/a,  A[i][k] <- A[i][k]/a,
//   A[i][j] <- A[i][j] - A[i][k] A[p][j] / a            (a = A[p][k], i != p, j != k).
// A pivot row keeps its values and records the factor -1/a in a per-row scale instead, so every
// lane runs the same update A[i][j] -= (A[i][k]/a) A[p][j] with the pivot row at scale 1 (a row
// is a pivot only once, before its scale changes).  After NP steps the window has turned once
// and x_k = sum_j A[p_k][j] y_{p_j}, i.e. M^{-1}[k][p_j] = scale(p_k) A[p_k][j]; written to Minv
// (LDS NP x NP, zero padded) with column q scaled by colscale[q].  brow: one LDS row of NP
// doubles of scratch.  Returns log|det M| = sum log|a_k|.
template <int NP>
__device__ __noinline__ double gj_inverse(int n, const DQMC_LDS double* M, DQMC_LDS double* Minv,
                                             const DQMC_LDS double* colscale, DQMC_LDS int* ordv,
                                             DQMC_LDS double* brow, int* flags) {
  const int i = threadIdx.x & 63;
  const int is = i < NP ? i : 0;
  double a[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) a[t] = (i < n) ? M[is * NP + t] : ((t == i) ? 1.0 : 0.0);
  bool used = (i >= NP);
  int myrank = -1, bad = 0;
  double scale = 1.0, mant = 1.0;
  int ex = 0;
  for (int k = 0; k < NP; ++k) {
    double amax;
    const int p = wave_argmax_lane(fabs(a[0]), !used, &amax);
    if (!(amax > 0.0)) bad = 1;
    const bool me = (i == p);
    if (me) row_store<NP>(brow, a);
    lds_order();
    const double piv = brow[0];
    const double inv = 1.0 / piv;
    int e1, e2;
    mant *= frexp(fabs(piv), &e1);
    mant = frexp(mant, &e2);
    ex += e1 + e2;
    const double f = me ? 0.0 : a[0] * inv;
    a[0] = a[1] - f * brow[1];
#pragma unroll
    for (int t = 2; t < NP; t += 2) {
      const dbl2 v = *(const DQMC_LDS dbl2*)(brow + t);
      a[t - 1] = a[t] - f * v.x;
      a[t] = a[t + 1] - f * v.y;
    }
    lds_order();
    a[NP - 1] = me ? -1.0 : f;
    if (me) { used = true; myrank = k; scale = -inv; }
    if (i == 0) ordv[k] = p;
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  if (i < NP && myrank >= 0) {
    if (myrank < n) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        if (j < n) {
          const int col = ordv[j];
          Minv[myrank * NP + col] = scale * a[j] * colscale[col];
        } else {
          Minv[myrank * NP + j] = 0.0;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) Minv[myrank * NP + j] = 0.0;
    }
  }
  if (bad && i == 0) atomicOr(flags, 8);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  return log(mant) + ex * 0.69314718055994530942;
}

}  // namespace stab
}  // namespace dqmc
