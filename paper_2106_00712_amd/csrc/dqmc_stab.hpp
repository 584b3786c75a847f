// Register-resident factorisations for the N <= 64 path: one wavefront per matrix, the matrix
// held in VGPRs (one column or one row per lane), the step loop unrolled at compile time so
// that every register index is static; pivots are chosen with a DPP wave maximum and a ballot,
// and pivot rows/columns move between lanes with v_readlane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqmc {
namespace stab {

#define DQMC_LDS __attribute__((address_space(3)))

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
  return b ? (int)__builtin_ctzll(b) : 0;
}

// Value of lane `lane` to every lane: BC = 0 through v_readlane (a scalar register), BC = 1
// through ds_bpermute (the LDS crossbar, asynchronous).
template <int BC>
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  if constexpr (BC == 0) return lane_read(v, lane);
  else return __shfl(v, lane);
}

// Column-pivoted Householder QR of the n x n block of X (LDS, NP x NP, zero padded) by one
// wavefront; lane c holds column c.  At step j the remaining column of largest norm over rows
// j..n-1 is the pivot p; its rows j.. are broadcast; every other remaining column c gets
// x_c -= beta (v^T x_c) v with v = x_p - alpha e_j, alpha = -sign(x_pj) |x_p|.
// Output: X overwritten in LAPACK form (R on and above the diagonal of the pivot order, v below;
// R[j][j] = alpha at column ordv[j]); vd[j] = v_j, bt[j] = beta_j, ordv[j] = pivot column,
// rank[c] = step of column c, dd[j] = |alpha_j|, sgn[j] = sign(alpha_j).
template <int NP, int BC>
__device__ __noinline__ void qr_factor(int n, DQMC_LDS double* X, DQMC_LDS double* vd,
                                       DQMC_LDS double* bt, DQMC_LDS int* rank,
                                       DQMC_LDS int* ordv, DQMC_LDS double* dd,
                                       DQMC_LDS double* sgn, int* flags) {
  const int c = threadIdx.x & 63;
  const int cs = c < NP ? c : 0;
  double x[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) x[r] = (c < n) ? X[r * NP + cs] : 0.0;
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < NP; ++r) nrm += x[r] * x[r];
  bool used = (c >= n);
  int myrank = -1;
  double myalpha = 0.0;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (j < n) {
      double nx2;
      const int p = wave_argmax_lane(nrm, !used, &nx2);
      double v[NP];
#pragma unroll
      for (int r = j; r < NP; ++r) v[r] = lane_bcast<BC>(x[r], p);
      const double xj = v[j];
      const double nx = sqrt(nx2);
      const double alpha = (xj >= 0.0) ? -nx : nx;
      const double beta = (nx > 0.0) ? 1.0 / (alpha * (alpha - xj)) : 0.0;
      const double v0 = xj - alpha;
      if (!(nx > 0.0)) bad = 1;
      if (c == p) { used = true; myrank = j; myalpha = alpha; }
      double w0 = v0 * x[j], w1 = 0.0;
#pragma unroll
      for (int r = j + 1; r < NP; ++r) {
        if ((r - j) & 1) w1 += v[r] * x[r]; else w0 += v[r] * x[r];
      }
      const double w = used ? 0.0 : (w0 + w1) * beta;
      x[j] -= w * v0;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int r = j + 1; r < NP; ++r) {
        x[r] -= w * v[r];
        if (r & 1) s1 += x[r] * x[r]; else s0 += x[r] * x[r];
      }
      nrm = s0 + s1;
      if (c == 0) {
        ordv[j] = p;
        vd[j] = v0;
        bt[j] = beta;
        dd[j] = fabs(alpha);
        sgn[j] = alpha < 0.0 ? -1.0 : 1.0;
      }
    }
  }
  if (c < NP) {
#pragma unroll
    for (int r = 0; r < NP; ++r) X[r * NP + c] = (r == myrank) ? myalpha : x[r];
    rank[c] = (c < n) ? myrank : -1;
  }
  if (bad && c == 0) atomicOr(flags, 8);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Q of the factorisation above, column jj = H_0 H_1 ... H_jj e_jj held by lane jj while the
// reflectors H_j (j descending) are applied; v_j is read from X (broadcast LDS loads).
// Writes U = Q Diag(sgn) to Ud (global NP x NP, zero padded).
template <int NP>
__device__ __noinline__ void qr_form_q(int n, const DQMC_LDS double* X, const DQMC_LDS double* vd,
                                       const DQMC_LDS double* bt, const DQMC_LDS int* ordv,
                                       const DQMC_LDS double* sgn, double* Ud) {
  const int c = threadIdx.x & 63;
  double q[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) q[r] = (r == c && c < n) ? 1.0 : 0.0;
#pragma unroll
  for (int j = NP - 1; j >= 0; --j) {
    if (j < n) {
      const int p = ordv[j];
      const double vj = vd[j], bj = bt[j];
      double w0 = vj * q[j], w1 = 0.0;
#pragma unroll
      for (int r = j + 1; r < NP; ++r) {
        const double vr = X[r * NP + p];
        if ((r - j) & 1) w1 += vr * q[r]; else w0 += vr * q[r];
      }
      const double w = (c >= j && c < n) ? (w0 + w1) * bj : 0.0;
      q[j] -= w * vj;
#pragma unroll
      for (int r = j + 1; r < NP; ++r) q[r] -= w * X[r * NP + p];
    }
  }
  if (c < NP) {
    const double s = (c < n) ? sgn[c] : 1.0;
#pragma unroll
    for (int r = 0; r < NP; ++r) Ud[r * NP + c] = q[r] * s;
  }
}

// In-place Gauss-Jordan inversion with implicit row pivoting (exchange steps) of the n x n
// block of M (LDS, NP x NP) by one wavefront; lane i holds row i.  Step k pivots on the
// remaining row p of largest |A[p][k]| and exchanges the roles of x_k and y_p in y = A x:
//   A[p][k] <- 1/a,  A[p][j] <- -A[p][j]/a,  A[i][k] <- A[i][k]/a,
//   A[i][j] <- A[i][j] - A[i][k] A[p][j] / a            (a = A[p][k], i != p, j != k).
// After all steps x_k = sum_j A[p_k][j] y_{p_j}, i.e. M^{-1}[k][p_j] = A[p_k][j]; that is
// written to Minv (LDS NP x NP, zero padded) with column q scaled by colscale[q], i.e.
// Minv <- M^{-1} Diag(colscale).  Returns log|det M| = sum log|a_k|.
template <int NP, int BC>
__device__ __noinline__ double gj_inverse(int n, const DQMC_LDS double* M, DQMC_LDS double* Minv,
                                          const DQMC_LDS double* colscale, DQMC_LDS int* ordv,
                                          int* flags) {
  const int i = threadIdx.x & 63;
  const int is = i < NP ? i : 0;
  double a[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) a[j] = (i < n) ? M[is * NP + j] : 0.0;
  bool used = (i >= n);
  int myrank = -1;
  double logabs = 0.0;
  int bad = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (k < n) {
      double amax;
      const int p = wave_argmax_lane(fabs(a[k]), !used, &amax);
      const double piv = lane_bcast<BC>(a[k], p);
      if (!(amax > 0.0)) bad = 1;
      logabs += log(fabs(piv));
      const double inv = 1.0 / piv;
      const bool me = (i == p);
      const double f = me ? 0.0 : a[k] * inv;
      // the pivot row travels in chunks of 16 so that only 16 of its values are live at once
#pragma unroll
      for (int j0 = 0; j0 < NP; j0 += 16) {
        double pr[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) pr[t] = lane_bcast<BC>(a[j0 + t], p);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int j = j0 + t;
          if (j == k) a[j] = me ? inv : f;
          else a[j] = me ? -a[j] * inv : a[j] - f * pr[t];
        }
      }
      if (me) { used = true; myrank = k; }
      if (i == 0) ordv[k] = p;
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  if (i < n) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      if (j < n) {
        const int col = ordv[j];
        Minv[myrank * NP + col] = a[j] * colscale[col];
      } else {
        Minv[myrank * NP + j] = 0.0;
      }
    }
  } else if (i < NP) {
#pragma unroll
    for (int j = 0; j < NP; ++j) Minv[i * NP + j] = 0.0;
  }
  if (bad && i == 0) atomicOr(flags, 8);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  return logabs;
}

}  // namespace stab
}  // namespace dqmc
