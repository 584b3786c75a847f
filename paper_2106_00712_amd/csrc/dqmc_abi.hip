// Host side of libdqmc.so: the C ABI declared in include/dqmc.h, the workspace layout, and the
// kernels that are not part of the per-chain sweep (model constants, measurements, probes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dqmc.h"
#include "dqmc_error.hpp"
#include "dqmc_device.hpp"
#include "dqmc_fast.hpp"
#include "dqmc_kernels.hpp"

using namespace dqmc;

namespace {

// The last error message of the calling thread, in a fixed buffer (setting it allocates nothing).
thread_local char g_err[512];

dqmc_status fail(dqmc_status s, const char* msg) {
  std::snprintf(g_err, sizeof g_err, "%s", msg);
  return s;
}
dqmc_status fail(dqmc_status s, const std::string& msg) { return fail(s, msg.c_str()); }

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      std::snprintf(g_err, sizeof g_err, "%s: %s", #expr, hipGetErrorString(e_));        \
      return DQMC_EDEVICE;                                                               \
    }                                                                                    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------------ model constants
// e^{A} for A = sign * (-dtau) (T - mu I) by scaling and squaring of the degree-18 Taylor
// polynomial (Horner form, one MFMA product per degree) on one workgroup:
//   E_18 = I,  E_{k-1} = I + (A / 2^s) E_k / k,  then E_0 squared s times.
// ||A / 2^s||_1 <= 1/2, so the truncation error is below 1e-22 relative.
constexpr int TAYLOR_DEGREE = 18;

__global__ __launch_bounds__(NT) void constants_kernel(int n, int np, double dtau, double mu, int s,
                                                      double* Tp, double* A, double* E0,
                                                      double* E1, double* expK, double* expKinv,
                                                      float* expK32, float* expKinv32, double* eye,
                                                      double* ones, int* err) {
  const int tid = threadIdx.x;
  if (tid == 0) *err = 0;
  for (int e = tid; e < np * np; e += NT) {
    int i = e / np, j = e - i * np;
    eye[e] = (i == j && i < n) ? 1.0 : 0.0;
  }
  for (int i = tid; i < np; i += NT) ones[i] = 1.0;
  // the hopping matrix arrives as its n x n block of the np x np array: zero the padding
  for (int e = tid; e < np * np; e += NT) {
    int i = e / np, j = e - i * np;
    if (!(i < n && j < n)) Tp[e] = 0.0;
  }
  const double scale = std::ldexp(dtau, -s);
  for (int pass = 0; pass < 2; ++pass) {
    const double sg = pass == 0 ? -1.0 : 1.0;   // e^{-dtau(T-mu)} then e^{+dtau(T-mu)}
    for (int e = tid; e < np * np; e += NT) {
      int i = e / np, j = e - i * np;
      double v = 0.0;
      if (i < n && j < n) v = sg * scale * (Tp[e] - (i == j ? mu : 0.0));
      A[e] = v;
      E0[e] = (i == j && i < n) ? 1.0 : 0.0;
    }
    __syncthreads();
    double* cur = E0;
    double* nxt = E1;
    for (int k = TAYLOR_DEGREE; k >= 1; --k) {
      const double ik = 1.0 / k;
      wg_gemm<double>(1, np, np, np, A, A, np, 1, cur, cur, np, 1, [&](int, int i, int j, double v) {
        nxt[i * np + j] = ((i == j && i < n) ? 1.0 : 0.0) + v * ik;
      });
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
    for (int q = 0; q < s; ++q) {
      wg_gemm<double>(1, np, np, np, cur, cur, np, 1, cur, cur, np, 1,
                      [&](int, int i, int j, double v) { nxt[i * np + j] = v; });
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
    double* dst = pass == 0 ? expK : expKinv;
    float* dst32 = pass == 0 ? expK32 : expKinv32;
    for (int e = tid; e < np * np; e += NT) {
      dst[e] = cur[e];
      dst32[e] = (float)cur[e];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------ measurements
// Equal-time estimators of one chain from its fresh G(0) (Wick's theorem at a fixed field):
// <n_i sigma> = 1 - G_ii, double occupancy (1/N) sum_i (1 - G^up_ii)(1 - G^dn_ii), density,
// kinetic energy (1/N) sum_sigma sum_ij T_ij (delta_ij - G_ji).
__global__ __launch_bounds__(NT) void measure_kernel(KArgs a, dqmc_obs* obs, double* green) {
  const int chain = blockIdx.x, tid = threadIdx.x;
  const int n = a.n, np = a.np;
  char* cb = a.base + (size_t)chain * a.stride;
  const ChainStats* st = (const ChainStats*)(cb + a.o_stats);
  const double* G64 = (const double*)(cb + a.o_G64);
  const double* Gu = G64;
  const double* Gd = G64 + (size_t)np * np;
  __shared__ double red[3][NW];
  double docc = 0, dens = 0, kin = 0;
  for (int i = tid; i < n; i += NT) {
    double gu = Gu[i * np + i], gd = Gd[i * np + i];
    docc += (1.0 - gu) * (1.0 - gd);
    dens += 2.0 - gu - gd;
  }
  for (int e = tid; e < n * n; e += NT) {
    int i = e / n, j = e - i * n;
    double t = a.Tm[i * np + j];
    if (t != 0.0) kin += t * (2.0 * (i == j ? 1.0 : 0.0) - Gu[j * np + i] - Gd[j * np + i]);
  }
  docc = wave_sum(docc);
  dens = wave_sum(dens);
  kin = wave_sum(kin);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = docc;
    red[1][tid >> 6] = dens;
    red[2][tid >> 6] = kin;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int w = 0; w < NW; ++w) { s0 += red[0][w]; s1 += red[1][w]; s2 += red[2][w]; }
    dqmc_obs o;
    o.double_occ = s0 / n;
    o.density = s1 / n;
    o.kinetic = s2 / n;
    o.logdet_up = st->logdet[0];
    o.logdet_dn = st->logdet[1];
    o.max_drift = st->max_drift;
    o.max_logdet_err = st->max_logdet_err;
    o.attempted = st->attempted;
    o.accepted = st->accepted;
    o.near_ties = st->near_ties;
    o.sweeps_done = st->sweeps_done;
    o.flags = st->flags;
    o.reserved = 0;
    o.slice_double_occ = st->slice_meas ? st->slice_docc / st->slice_meas : 0.0;
    o.slice_kinetic = st->slice_meas ? st->slice_kin / st->slice_meas : 0.0;
    o.slice_meas = st->slice_meas;
    obs[chain] = o;
  }
  if (green) {
    double* out = green + (size_t)chain * 2 * n * n;
    for (int e = tid; e < 2 * n * n; e += NT) {
      int sp = e / (n * n), i = (e / n) % n, j = e % n;
      out[e] = G64[(size_t)sp * np * np + i * np + j];
    }
  }
}

// (1/N) sum_ij f_i f_j <s^z_i s^z_j> at G(0) by Wick's theorem (both spins independent at a fixed
// field): (1/(4N)) [m^2 + sum_s (sum_i f_i^2 G^s_ii - sum_ij f_i f_j G^s_ij G^s_ji)] with
// m = sum_i f_i (G^dn_ii - G^up_ii).  One block per chain.
__global__ __launch_bounds__(NT) void spin_structure_kernel(KArgs a, const double* form, double* out) {
  const int chain = blockIdx.x, tid = threadIdx.x;
  const int n = a.n, np = a.np;
  const double* G64 = (const double*)(a.base + (size_t)chain * a.stride + a.o_G64);
  __shared__ double red[2][NW];
  double m = 0, acc = 0;
  for (int i = tid; i < n; i += NT) {
    double f = form[i], gu = G64[i * np + i], gd = G64[(size_t)np * np + i * np + i];
    m += f * (gd - gu);
    acc += f * f * (gu + gd);
  }
  for (int e = tid; e < n * n; e += NT) {
    int i = e / n, j = e - i * n;
    double ff = form[i] * form[j];
    if (ff == 0.0) continue;
    for (int sp = 0; sp < 2; ++sp) {
      const double* G = G64 + (size_t)sp * np * np;
      acc -= ff * G[i * np + j] * G[j * np + i];
    }
  }
  m = wave_sum(m);
  acc = wave_sum(acc);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = m;
    red[1][tid >> 6] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double sm = 0, sa = 0;
    for (int w = 0; w < NW; ++w) { sm += red[0][w]; sa += red[1][w]; }
    out[chain] = (sm * sm + sa) / (4.0 * n);
  }
}

// Row s of a per-sweep series: every chain's estimators at its fresh G(0), computed exactly as
// measure_kernel (double occupancy, density, kinetic energy) and spin_structure_kernel (the
// structure factor of form, 0 without one) compute them: same loops, same summation order.
__global__ __launch_bounds__(NT) void series_kernel(KArgs a, const double* form, double* series, int s) {
  const int chain = blockIdx.x, tid = threadIdx.x;
  const int n = a.n, np = a.np;
  const double* G64 = (const double*)(a.base + (size_t)chain * a.stride + a.o_G64);
  const double* Gu = G64;
  const double* Gd = G64 + (size_t)np * np;
  __shared__ double red[5][NW];
  double docc = 0, dens = 0, kin = 0, m = 0, acc = 0;
  for (int i = tid; i < n; i += NT) {
    double gu = Gu[i * np + i], gd = Gd[i * np + i];
    docc += (1.0 - gu) * (1.0 - gd);
    dens += 2.0 - gu - gd;
  }
  for (int e = tid; e < n * n; e += NT) {
    int i = e / n, j = e - i * n;
    double t = a.Tm[i * np + j];
    if (t != 0.0) kin += t * (2.0 * (i == j ? 1.0 : 0.0) - Gu[j * np + i] - Gd[j * np + i]);
  }
  if (form) {
    for (int i = tid; i < n; i += NT) {
      double f = form[i], gu = Gu[i * np + i], gd = Gd[i * np + i];
      m += f * (gd - gu);
      acc += f * f * (gu + gd);
    }
    for (int e = tid; e < n * n; e += NT) {
      int i = e / n, j = e - i * n;
      double ff = form[i] * form[j];
      if (ff == 0.0) continue;
      for (int sp = 0; sp < 2; ++sp) {
        const double* G = G64 + (size_t)sp * np * np;
        acc -= ff * G[i * np + j] * G[j * np + i];
      }
    }
  }
  docc = wave_sum(docc);
  dens = wave_sum(dens);
  kin = wave_sum(kin);
  m = wave_sum(m);
  acc = wave_sum(acc);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = docc;
    red[1][tid >> 6] = dens;
    red[2][tid >> 6] = kin;
    red[3][tid >> 6] = m;
    red[4][tid >> 6] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0, s1 = 0, s2 = 0, sm = 0, sa = 0;
    for (int w = 0; w < NW; ++w) {
      s0 += red[0][w]; s1 += red[1][w]; s2 += red[2][w]; sm += red[3][w]; sa += red[4][w];
    }
    double* dst = series + ((size_t)s * a.n_chains + chain) * DQMC_SERIES_WIDTH;
    dst[0] = s0 / n;
    dst[1] = s1 / n;
    dst[2] = s2 / n;
    dst[3] = form ? (sm * sm + sa) / (4.0 * n) : 0.0;
  }
}

// OR of every chain's flags (obs[0 .. n_chains)) into *out; one block.
__global__ __launch_bounds__(NT) void flags_or_kernel(const dqmc_obs* obs, int n_chains, int* out) {
  __shared__ int acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  int f = 0;
  for (int c = threadIdx.x; c < n_chains; c += NT) f |= obs[c].flags;
  if (f) atomicOr(&acc, f);
  __syncthreads();
  if (threadIdx.x == 0) *out = acc;
}

__global__ void get_fields_kernel(KArgs a, int8_t* out) {
  const int chain = blockIdx.x;
  const int8_t* f = (const int8_t*)(a.base + (size_t)chain * a.stride + a.o_fields);
  for (int e = threadIdx.x; e < a.L * a.n; e += blockDim.x) {
    int l = e / a.n, i = e - l * a.n;
    out[(size_t)chain * a.L * a.n + e] = f[l * a.np + i];
  }
}

__global__ void copy_propagators_kernel(KArgs a) {
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < 2 * a.n * a.n; e += blockDim.x * gridDim.x) {
    int w = e / (a.n * a.n), i = (e / a.n) % a.n, j = e % a.n;
    a.out[e] = (w ? a.expKinv : a.expK)[i * a.np + j];
  }
}

__global__ void phase_ticks_kernel(KArgs a, int64_t* out) {
  int chain = blockIdx.x * blockDim.x + threadIdx.x;
  if (chain >= a.n_chains) return;
  const ChainStats* st = (const ChainStats*)(a.base + (size_t)chain * a.stride + a.o_stats);
  for (int k = 0; k < 16; ++k) out[(size_t)chain * 16 + k] = st->ticks[k];
}

__global__ void philox_kernel(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                              uint64_t c3, int n_blocks, uint64_t* out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_blocks) return;
  u64x4 w = philox4x64_10(u64x4{c0 + (uint64_t)j, c1, c2, c3}, k0, k1);
  out[4 * j + 0] = w.x0;
  out[4 * j + 1] = w.x1;
  out[4 * j + 2] = w.x2;
  out[4 * j + 3] = w.x3;
}

// One wave: C = A B for a 16x4 A and a 4x16 B, written through the layout the library assumes.
__global__ void mfma_probe_kernel(const double* a64, const double* b64, double* out64,
                                  const float* a32, const float* b32, float* out32) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc = {0, 0, 0, 0};
  acc = mfma(a64[li * 4 + lk], b64[lk * 16 + li], acc);
  f4 acc32 = {0, 0, 0, 0};
  acc32 = mfma(a32[li * 4 + lk], b32[lk * 16 + li], acc32);
  for (int v = 0; v < 4; ++v) {
    out64[out_row<double>(v, lane) * 16 + li] = acc[v];
    out32[out_row<float>(v, lane) * 16 + li] = acc32[v];
  }
}

}  // namespace

// ------------------------------------------------------------------------ the handle
struct dqmc_batch {
  int n, np, L, stab, J, K, n_chains, precision;
  bool small, fast;
  size_t lds_bytes, fast_lds_bytes;
  KArgs args;   // base arguments (op fields filled per call)
  char* ws;
  size_t ws_bytes;
  size_t c_seeds, c_slots, c_err;   // staging areas in the workspace
};

struct dqmc_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<KArgs> args;
  ~dqmc_graph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

namespace {

struct Layout {
  int n, np, L, stab, J, K, precision;
  bool small, fast;
  size_t lds_bytes, fast_lds_bytes;
  // constants region (offsets from the workspace base)
  size_t c_expK, c_expKinv, c_expK32, c_expKinv32, c_T, c_eye, c_ones, c_A, c_E0, c_E1, c_seeds,
      c_slots, c_err, c_end;
  // per chain
  size_t o_stats, o_fields, o_G64, o_stack, o_left, o_Gw, o_work, o_xy, o_qrv, o_lstack, stride;
  int KT;   // accumulated delayed-update rank (workspace variant), 0 otherwise
};

int max_lds_per_block() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      cached = v;
    else
      cached = 160 * 1024;
  }
  return cached;
}

dqmc_status make_layout(const dqmc_model* m, int32_t n_chains, Layout* out, bool query_device) {
  if (!m) return fail(DQMC_EINVAL, "model is NULL");
  if (m->n_sites < 1 || m->n_sites > 2048) return fail(DQMC_EINVAL, "n_sites must be in [1, 2048]");
  if (m->n_slices < 1) return fail(DQMC_EINVAL, "n_slices must be >= 1");
  if (!(m->dtau > 0.0) || !(m->U >= 0.0) || !std::isfinite(m->mu))
    return fail(DQMC_EINVAL, "need dtau > 0, U >= 0, finite mu");
  if (m->stab_every < 1) return fail(DQMC_EINVAL, "stab_every must be >= 1");
  if (m->precision != DQMC_FP64 && m->precision != DQMC_FP32_WRAP)
    return fail(DQMC_EINVAL, "unknown precision");
  if (m->refresh_every < 0 || m->delay_rank < 0) return fail(DQMC_EINVAL, "negative refresh/delay");
  if (m->qr_blocked != 0 && m->qr_blocked != 1) return fail(DQMC_EINVAL, "qr_blocked must be 0 or 1");
  if (m->sweep_mode < 0 || m->sweep_mode > 3) return fail(DQMC_EINVAL, "sweep_mode must be in [0, 3]");
  if (!(m->drift_limit >= 0.0) || !std::isfinite(m->drift_limit))
    return fail(DQMC_EINVAL, "drift_limit must be finite and >= 0");
  if (n_chains < 0) return fail(DQMC_EINVAL, "n_chains must be >= 0");
  Layout L{};
  L.n = m->n_sites;
  // padded size: a multiple of 16; up to 64 sites the padded sizes of the register/LDS sweep
  // kernels (16, 32, 64)
  L.np = L.n <= 16 ? 16 : L.n <= 32 ? 32 : L.n <= 64 ? 64 : (L.n + 15) & ~15;
  L.L = m->n_slices;
  L.precision = m->precision;
  int stab = m->stab_every;
  if (m->precision == DQMC_FP32_WRAP && m->refresh_every > 0) stab = std::min(stab, m->refresh_every);
  L.stab = std::min(stab, L.L);
  L.J = (L.L + L.stab - 1) / L.stab;
  const size_t wts = m->precision == DQMC_FP32_WRAP ? sizeof(float) : sizeof(double);
  const size_t nn = (size_t)L.np * L.np;
  // delay rank: multiple of 4; the small variant stores the panels in its work matrices.  Default
  // 16, and 32 from N = 128 on, where the flush (a pass over G in HBM per block) dominates
  int kreq = m->delay_rank > 0 ? m->delay_rank : (L.n >= 128 ? 32 : 16);
  kreq = (kreq + 3) & ~3;
  const int lds_limit = query_device ? max_lds_per_block() : 160 * 1024;
  auto small_bytes = [&](int K) {
    return (wts == 8 ? lds_mat_bytes<double>(L.np) : lds_mat_bytes<float>(L.np)) +
           lds_vec_doubles(L.np, K) * sizeof(double);
  };
  int k_small = std::min(kreq, 16);
  k_small = std::min(k_small, (int)(wts == 8 ? L.np / 2 : L.np));
  k_small = std::max(4, k_small & ~3);
  // the sweep modes (alternating sweeps, per-slice measurements) run in the workspace kernels
  L.small = m->sweep_mode == 0 && small_bytes(k_small) <= (size_t)lds_limit;
  if (L.small) {
    L.K = k_small;
    L.lds_bytes = small_bytes(L.K);
  } else {
    L.K = std::max(4, std::min(kreq, 32));
    L.lds_bytes = (lds_vec_doubles(L.np, L.K) + TG_STAGE_DOUBLES) * sizeof(double);
    if (L.lds_bytes > (size_t)lds_limit) return fail(DQMC_EINVAL, "n_sites too large for LDS vectors");
  }
  // fast sweep path: padded size 16, 32 or 64, block size 8 or 16 sites
  L.fast = false;
  L.fast_lds_bytes = 0;
  if (m->sweep_mode == 0 && (L.np == 16 || L.np == 32 || L.np == 64)) {
    const int kb = (kreq <= 8 || L.np == 16) ? 8 : 16;
    size_t fb = 0;
    const bool f32 = wts == 4;
#define DQMC_FB(NPV, KBV) (f32 ? fast::Fast<NPV, float, KBV>::lds_bytes() : fast::Fast<NPV, double, KBV>::lds_bytes())
    if (L.np == 16) fb = DQMC_FB(16, 8);
    else if (L.np == 32) fb = kb == 8 ? DQMC_FB(32, 8) : DQMC_FB(32, 16);
    else fb = kb == 8 ? DQMC_FB(64, 8) : DQMC_FB(64, 16);
#undef DQMC_FB
    if (fb <= (size_t)lds_limit) {
      L.fast = true;
      L.fast_lds_bytes = fb;
      L.K = kb;   // one block size for both kernels, so that init/debug and sweeps agree
      if (L.small) L.lds_bytes = small_bytes(L.K);
      if (L.lds_bytes > (size_t)lds_limit) return fail(DQMC_EINVAL, "LDS budget exceeded");
    }
  }
  // constants
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.c_expK = take(nn * 8);
  L.c_expKinv = take(nn * 8);
  L.c_expK32 = take(nn * 4);
  L.c_expKinv32 = take(nn * 4);
  L.c_T = take(nn * 8);
  L.c_eye = take(nn * 8);
  L.c_ones = take((size_t)L.np * 8);
  L.c_A = take(nn * 8);
  L.c_E0 = take(nn * 8);
  L.c_E1 = take(nn * 8);
  L.c_seeds = take((size_t)std::max(n_chains, 1) * 8);
  L.c_slots = take((size_t)std::max(n_chains, 1) * 4);
  L.c_err = take(256);
  L.c_end = off;
  // chain
  size_t co = 0;
  auto ctake = [&](size_t bytes) { size_t o = co; co = align256(co + bytes); return o; };
  L.o_stats = ctake(sizeof(ChainStats));
  L.o_fields = ctake((size_t)L.L * L.np);
  L.o_G64 = ctake(2 * nn * 8);
  L.o_stack = ctake(2 * (size_t)L.J * (2 * nn + L.np) * 8);
  L.o_left = ctake(2 * (3 * nn + L.np) * 8);
  L.o_Gw = ctake(2 * nn * 8);   // working G of the global variant / parked G of the fast path
  if (!L.small) {
    L.o_work = ctake(2 * nn * 8);
    // two-level delayed updates from N = 128 on (below, the correction products cost more than
    // the flushes they save): panels XA, YA of rank KT = 4K for both spins, the corrected columns
    // and rows of one block, and the gathered panel rows and columns
    L.KT = (L.n >= 128) ? 4 * L.K : 0;
    const size_t K16 = (L.K + 15) & ~15;
    L.o_xy = L.KT ? ctake((4 * (size_t)L.np * L.KT + 4 * (size_t)L.np * K16 + 4 * (size_t)L.KT * K16) * wts)
                  : ctake(4 * (size_t)L.np * L.K * wts);
    // blocked factorisations (np <= QR_BLOCK_MAX_NP): QR reflectors (np x np) and one QB x QB
    // T per panel; the Gauss-Jordan solve reuses the area for its np x QB and QB x 2np panels
    // (3 QB np doubles, more than the QR's np^2 + QB np below np = 2 QB)
    L.o_qrv = (L.np <= QR_BLOCK_MAX_NP)
                  ? ctake(std::max(nn + (size_t)QB * L.np, 3 * (size_t)QB * L.np) * 8) : 0;
    // left UDT stack of the alternating sweeps, laid out like the right stack
    L.o_lstack = (m->sweep_mode & 1) ? ctake(2 * (size_t)L.J * (2 * nn + L.np) * 8) : 0;
  } else {
    L.o_work = L.o_xy = L.o_qrv = L.o_lstack = 0;
    L.KT = 0;
  }
  L.stride = align256(co);
  *out = L;
  return DQMC_OK;
}

void fill_args(const Layout& L, const dqmc_model* m, char* ws, int n_chains, KArgs* a) {
  std::memset(a, 0, sizeof(*a));
  a->n = L.n; a->np = L.np; a->L = L.L; a->stab = L.stab; a->J = L.J; a->K = L.K;
  a->KT = L.KT;
  a->n_chains = n_chains;
  const double nu = std::acosh(std::exp(0.5 * m->U * m->dtau));
  a->nu = nu;
  a->ev[0] = std::exp(nu);
  a->ev[1] = std::exp(-nu);
  a->dup[0] = std::exp(2.0 * nu) - 1.0;    // s = -1: e^{-2 nu s} - 1
  a->dup[1] = std::exp(-2.0 * nu) - 1.0;   // s = +1
  a->ddn[0] = std::exp(-2.0 * nu) - 1.0;   // s = -1: e^{+2 nu s} - 1
  a->ddn[1] = std::exp(2.0 * nu) - 1.0;
  a->drift_limit = m->drift_limit > 0.0 ? m->drift_limit : (m->precision == DQMC_FP32_WRAP ? 1e-5 : 1e-3);
  a->expK = (const double*)(ws + L.c_expK);
  a->expKinv = (const double*)(ws + L.c_expKinv);
  a->expK32 = (const float*)(ws + L.c_expK32);
  a->expKinv32 = (const float*)(ws + L.c_expKinv32);
  a->Tm = (const double*)(ws + L.c_T);
  a->eye = (const double*)(ws + L.c_eye);
  a->ones = (const double*)(ws + L.c_ones);
  a->err = (int*)(ws + L.c_err);
  a->base = ws + L.c_end;
  a->stride = L.stride;
  a->o_fields = L.o_fields; a->o_G64 = L.o_G64; a->o_Gw = L.o_Gw; a->o_stack = L.o_stack;
  a->o_left = L.o_left; a->o_work = L.o_work; a->o_xy = L.o_xy; a->o_stats = L.o_stats;
  a->o_qrv = L.o_qrv;
  a->o_lstack = L.o_lstack;
  a->sweep_mode = m->sweep_mode;
  a->qr_blocked = m->qr_blocked;
}

// The kernel a batch runs for an operation, and its LDS bytes.
KernelRef fast_ref(const dqmc_batch* b) {
  const bool f32 = b->precision == DQMC_FP32_WRAP;
  if (b->np == 16) return f32 ? fast_kernel_f32_np16(b->K) : fast_kernel_f64_np16(b->K);
  if (b->np == 32) return f32 ? fast_kernel_f32_np32(b->K) : fast_kernel_f64_np32(b->K);
  return f32 ? fast_kernel_f32_np64(b->K) : fast_kernel_f64_np64(b->K);
}

KernelRef resolve(const dqmc_batch* b, int op) {
  const bool f32 = b->precision == DQMC_FP32_WRAP;
  if (op == OP_SWEEP && b->fast) return fast_ref(b);
  const void* fn = f32 ? (b->small ? chain_kernel_f32_lds() : chain_kernel_f32_ws())
                       : (b->small ? chain_kernel_f64_lds() : chain_kernel_f64_ws());
  return {fn, b->lds_bytes};
}

dqmc_status prepare(const KernelRef& k) {
  if (k.lds > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.lds));
  return DQMC_OK;
}

// One workgroup of NT threads per chain (or per listed slot).
dqmc_status launch(const dqmc_batch* b, const KArgs& a, hipStream_t s, int grid = -1) {
  if (grid < 0) grid = b->n_chains;
  if (grid == 0) return DQMC_OK;
  const KernelRef k = resolve(b, a.op);
  dqmc_status st = prepare(k);
  if (st != DQMC_OK) return st;
  KArgs arg = a;
  void* params[] = {&arg};
  HIP_TRY(hipLaunchKernel(k.fn, dim3(grid), dim3(NT), params, k.lds, s));
  return DQMC_OK;
}

// Side streams for sweeping several batches at once, created on first use and kept for the
// life of the process (default priority, non-blocking).
struct SidePool {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipEvent_t fork = nullptr;
  dqmc_status grow(int n) {
    if (!fork && hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess)
      return fail(DQMC_EDEVICE, "side pool: event");
    while ((int)streams.size() < n) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return fail(DQMC_EDEVICE, "side pool: stream");
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        hipStreamDestroy(st);
        return fail(DQMC_EDEVICE, "side pool: event");
      }
      streams.push_back(st);
      events.push_back(ev);
    }
    return DQMC_OK;
  }
};

SidePool& side_pool() {
  static thread_local SidePool pool;
  return pool;
}

}  // namespace

namespace {

// Everything dqmc_init_chains does once the layout is known and the workspace is checked: the
// model constants, the chains' fields, seeds and initial Green's functions.  Fills *b (the
// caller's storage) and waits for its work; allocates nothing.
dqmc_status init_core(dqmc_batch* b, const Layout& L, const dqmc_model* m, int32_t n_chains,
                      const int8_t* fields, const uint64_t* seeds, char* ws, size_t ws_bytes,
                      hipStream_t s) {
  if (!m->hopping) return fail(DQMC_EINVAL, "hopping is NULL");
  if (n_chains > 0 && !seeds) return fail(DQMC_EINVAL, "seeds is NULL");
  double norm1 = 0.0;
  for (int j = 0; j < L.n; ++j) {
    double col = 0.0;
    for (int i = 0; i < L.n; ++i) {
      const double t = m->hopping[i * L.n + j];
      if (!std::isfinite(t) || t != m->hopping[j * L.n + i])
        return fail(DQMC_EINVAL, "hopping must be finite and symmetric");
      col += std::fabs(m->dtau * (t - (i == j ? m->mu : 0.0)));
    }
    norm1 = std::max(norm1, col);
  }
  int sq = 0;
  while (std::ldexp(norm1, -sq) > 0.5) ++sq;
  // the n x n hopping block into the np x np array (the constants kernel zeroes the padding)
  HIP_TRY(hipMemcpy2DAsync(ws + L.c_T, (size_t)L.np * 8, m->hopping, (size_t)L.n * 8, (size_t)L.n * 8,
                           (size_t)L.n, hipMemcpyHostToDevice, s));
  if (n_chains > 0)
    HIP_TRY(hipMemcpyAsync(ws + L.c_seeds, seeds, (size_t)n_chains * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(constants_kernel, dim3(1), dim3(NT), 0, s, L.n, L.np, m->dtau, m->mu, sq,
                     (double*)(ws + L.c_T), (double*)(ws + L.c_A), (double*)(ws + L.c_E0),
                     (double*)(ws + L.c_E1), (double*)(ws + L.c_expK), (double*)(ws + L.c_expKinv),
                     (float*)(ws + L.c_expK32), (float*)(ws + L.c_expKinv32),
                     (double*)(ws + L.c_eye), (double*)(ws + L.c_ones), (int*)(ws + L.c_err));
  HIP_TRY(hipGetLastError());
  b->n = L.n; b->np = L.np; b->L = L.L; b->stab = L.stab; b->J = L.J; b->K = L.K;
  b->n_chains = n_chains; b->precision = L.precision; b->small = L.small; b->lds_bytes = L.lds_bytes;
  b->fast = L.fast; b->fast_lds_bytes = L.fast_lds_bytes;
  b->ws = ws; b->ws_bytes = ws_bytes;
  b->c_seeds = L.c_seeds; b->c_slots = L.c_slots; b->c_err = L.c_err;
  fill_args(L, m, ws, n_chains, &b->args);
  KArgs a = b->args;
  a.op = OP_INIT;
  a.gen_fields = fields ? 0 : 1;
  a.fields_in = fields;
  a.seeds = (const uint64_t*)(ws + L.c_seeds);
  dqmc_status st = launch(b, a, s);
  if (st != DQMC_OK) return st;
  int err = 0;
  HIP_TRY(hipMemcpyAsync(&err, ws + L.c_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err) return fail(DQMC_EINVAL, "fields must be +1 or -1");
  return DQMC_OK;
}

}  // namespace

// ------------------------------------------------------------------------ static workspace
// The chains' state of dqmc_run_static: a file-scope device array, one copy per GPU, held until
// the process ends.  In host code its name is not a device address: the address comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that address
// (rounded up to 256 bytes, the workspace alignment; the array has 256 bytes of slack for it) is
// passed to kernels and copies.  The runtime finds a device variable by its name among the code
// object's exported symbols, so the array has external linkage (an internal-linkage array is a
// local symbol there, which hipGetSymbolAddress cannot resolve); "used": no device code names it.
__device__ __attribute__((used, aligned(256))) char dqmc_static_scratch[DQMC_STATIC_BYTES + 256];

namespace {

constexpr int MAX_DEVICES = 64;
std::atomic<char*> g_scratch[MAX_DEVICES];

// Device address of the current device's copy of dqmc_static_scratch.
dqmc_status scratch_ptr(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DQMC_EDEVICE, "device index out of range");
  char* p = g_scratch[dev].load();
  if (!p) {
    void* q = nullptr;
    HIP_TRY(hipGetSymbolAddress(&q, HIP_SYMBOL(dqmc_static_scratch)));
    if (!q) return fail(DQMC_EDEVICE, "hipGetSymbolAddress(dqmc_static_scratch) gave NULL");
    p = (char*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    g_scratch[dev].store(p);
  }
  *out = p;
  return DQMC_OK;
}

}  // namespace

// Error message shared with the other translation units of the library (dqmc_last_error).
dqmc_status dqmc::set_error(dqmc_status s, const std::string& msg) { return fail(s, msg); }

// ------------------------------------------------------------------------ C ABI
extern "C" {

const char* dqmc_last_error(void) { return g_err; }

size_t dqmc_chain_bytes(const dqmc_model* m) {
  Layout L;
  if (make_layout(m, 1, &L, false) != DQMC_OK) return 0;
  return L.stride;
}

size_t dqmc_workspace_bytes(const dqmc_model* m, int32_t n_chains) {
  Layout L;
  if (make_layout(m, n_chains, &L, false) != DQMC_OK) return 0;
  return L.c_end + (size_t)n_chains * L.stride;
}

dqmc_status dqmc_init_chains(dqmc_batch** out, const dqmc_model* m, int32_t n_chains,
                             const int8_t* fields, const uint64_t* seeds, void* workspace,
                             size_t ws_bytes, void* stream) {
  if (!out) return fail(DQMC_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  dqmc_status st = make_layout(m, n_chains, &L, true);
  if (st != DQMC_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(DQMC_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = L.c_end + (size_t)n_chains * L.stride;
  if (ws_bytes < need) return fail(DQMC_ENOMEM, "workspace too small: need " + std::to_string(need));
  dqmc_batch* b = new (std::nothrow) dqmc_batch;
  if (!b) return fail(DQMC_EDEVICE, "host allocation failed");
  st = init_core(b, L, m, n_chains, fields, seeds, (char*)workspace, ws_bytes, (hipStream_t)stream);
  if (st != DQMC_OK) {
    delete b;
    return st;
  }
  *out = b;
  return DQMC_OK;
}

dqmc_status dqmc_sweep(dqmc_batch* b, int32_t n_sweeps, void* stream) {
  if (!b) return fail(DQMC_EINVAL, "batch is NULL");
  if (n_sweeps < 0) return fail(DQMC_EINVAL, "n_sweeps must be >= 0");
  if (n_sweeps == 0) return DQMC_OK;
  KArgs a = b->args;
  a.op = OP_SWEEP;
  a.n_sweeps = n_sweeps;
  return launch(b, a, (hipStream_t)stream);
}

// One sweep launch and one series launch per sweep, all enqueued on the stream back to back (no
// host synchronisation); consecutive one-sweep launches continue the chains exactly as one launch
// of n_sweeps would (the random numbers are indexed by each chain's global sweep counter).
dqmc_status dqmc_sweep_series(dqmc_batch* b, int32_t n_sweeps, const double* form, double* series,
                              void* stream) {
  if (!b || !series) return fail(DQMC_EINVAL, "batch/series is NULL");
  if (n_sweeps < 0) return fail(DQMC_EINVAL, "n_sweeps must be >= 0");
  if (n_sweeps == 0 || b->n_chains == 0) return DQMC_OK;
  hipStream_t s = (hipStream_t)stream;
  KArgs a = b->args;
  a.op = OP_SWEEP;
  a.n_sweeps = 1;
  for (int k = 0; k < n_sweeps; ++k) {
    dqmc_status st = launch(b, a, s);
    if (st != DQMC_OK) return st;
    hipLaunchKernelGGL(series_kernel, dim3(b->n_chains), dim3(NT), 0, s, b->args, form, series, k);
    HIP_TRY(hipGetLastError());
  }
  return DQMC_OK;
}

dqmc_status dqmc_sweep_multi(dqmc_batch* const* bs, const int32_t* n_sweeps, int32_t n, void* stream) {
  if (n < 0 || (n > 0 && (!bs || !n_sweeps))) return fail(DQMC_EINVAL, "bad batch list");
  for (int i = 0; i < n; ++i)
    if (!bs[i] || n_sweeps[i] < 0) return fail(DQMC_EINVAL, "bad batch entry");
  hipStream_t s = (hipStream_t)stream;
  if (n == 1) return dqmc_sweep(bs[0], n_sweeps[0], stream);
  if (n == 0) return DQMC_OK;
  // fork: every batch on a side stream after an event on the caller's stream, then join
  SidePool& P = side_pool();
  dqmc_status st = P.grow(n);
  if (st != DQMC_OK) return st;
  HIP_TRY(hipEventRecord(P.fork, s));
  for (int i = 0; i < n; ++i) {
    HIP_TRY(hipStreamWaitEvent(P.streams[i], P.fork, 0));
    st = dqmc_sweep(bs[i], n_sweeps[i], P.streams[i]);
    if (st != DQMC_OK) return st;
    HIP_TRY(hipEventRecord(P.events[i], P.streams[i]));
    HIP_TRY(hipStreamWaitEvent(s, P.events[i], 0));
  }
  return DQMC_OK;
}

dqmc_status dqmc_init_slots(dqmc_batch* b, const int32_t* slots, int32_t n_slots, const int8_t* fields,
                            const uint64_t* seeds, void* stream) {
  if (!b) return fail(DQMC_EINVAL, "batch is NULL");
  if (n_slots < 0 || n_slots > b->n_chains) return fail(DQMC_EINVAL, "n_slots out of range");
  if (n_slots == 0) return DQMC_OK;
  if (!slots || !seeds) return fail(DQMC_EINVAL, "slots/seeds is NULL");
  std::vector<char> seen(b->n_chains, 0);
  for (int i = 0; i < n_slots; ++i) {
    if (slots[i] < 0 || slots[i] >= b->n_chains) return fail(DQMC_EINVAL, "slot out of range");
    if (seen[slots[i]]++) return fail(DQMC_EINVAL, "slot listed twice");
  }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemsetAsync(b->ws + b->c_err, 0, sizeof(int), s));
  HIP_TRY(hipMemcpyAsync(b->ws + b->c_seeds, seeds, (size_t)n_slots * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->ws + b->c_slots, slots, (size_t)n_slots * 4, hipMemcpyHostToDevice, s));
  KArgs a = b->args;
  a.op = OP_INIT;
  a.gen_fields = fields ? 0 : 1;
  a.fields_in = fields;
  a.seeds = (const uint64_t*)(b->ws + b->c_seeds);
  a.slots = (const int32_t*)(b->ws + b->c_slots);
  dqmc_status st = launch(b, a, s, n_slots);
  if (st != DQMC_OK) return st;
  int err = 0;
  HIP_TRY(hipMemcpyAsync(&err, b->ws + b->c_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err) return fail(DQMC_EINVAL, "fields must be +1 or -1");
  return DQMC_OK;
}

dqmc_status dqmc_sweep_counts(dqmc_batch* b, const int32_t* counts, void* stream) {
  if (!b || !counts) return fail(DQMC_EINVAL, "batch/counts is NULL");
  KArgs a = b->args;
  a.op = OP_SWEEP;
  a.n_sweeps = 0;
  a.counts = counts;
  return launch(b, a, (hipStream_t)stream);
}

dqmc_status dqmc_measure(dqmc_batch* b, dqmc_obs* obs, double* green, void* stream) {
  if (!b || !obs) return fail(DQMC_EINVAL, "batch/obs is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (b->n_chains == 0) return DQMC_OK;
  hipLaunchKernelGGL(measure_kernel, dim3(b->n_chains), dim3(NT), 0, s, b->args, obs, green);
  HIP_TRY(hipGetLastError());
  std::vector<dqmc_obs> h(b->n_chains);
  HIP_TRY(hipMemcpyAsync(h.data(), obs, h.size() * sizeof(dqmc_obs), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (const dqmc_obs& o : h)
    if (o.flags) return fail(DQMC_ENUMERIC, "a chain raised a numerical flag");
  return DQMC_OK;
}

dqmc_status dqmc_spin_structure(dqmc_batch* b, const double* form, double* out, void* stream) {
  if (!b || !form || !out) return fail(DQMC_EINVAL, "batch/form/out is NULL");
  if (b->n_chains == 0) return DQMC_OK;
  hipLaunchKernelGGL(spin_structure_kernel, dim3(b->n_chains), dim3(NT), 0, (hipStream_t)stream,
                     b->args, form, out);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_get_fields(dqmc_batch* b, int8_t* out, void* stream) {
  if (!b || !out) return fail(DQMC_EINVAL, "batch/out is NULL");
  if (b->n_chains == 0) return DQMC_OK;
  hipLaunchKernelGGL(get_fields_kernel, dim3(b->n_chains), dim3(256), 0, (hipStream_t)stream,
                     b->args, out);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_destroy(dqmc_batch* b) {
  delete b;
  return DQMC_OK;
}

dqmc_status dqmc_batch_info(const dqmc_batch* b, int32_t* k, int32_t* stab, int32_t* lds_bytes,
                            int32_t* variant) {
  if (!b) return fail(DQMC_EINVAL, "batch is NULL");
  if (k) *k = b->K;
  if (stab) *stab = b->stab;
  if (lds_bytes) *lds_bytes = (int32_t)(b->fast ? b->fast_lds_bytes : b->lds_bytes);
  if (variant) *variant = b->fast ? 2 : (b->small ? 0 : 1);
  return DQMC_OK;
}

dqmc_status dqmc_debug_green(dqmc_batch* b, int32_t slice, int32_t n_wraps, double* out, void* stream) {
  if (!b || !out) return fail(DQMC_EINVAL, "batch/out is NULL");
  if (slice < 0 || slice > b->L || slice + n_wraps < 0 || slice + n_wraps > b->L)
    return fail(DQMC_EINVAL, "slice range");
  KArgs a = b->args;
  a.op = OP_DEBUG_GREEN;
  a.slice = slice;
  a.n_wraps = n_wraps;
  a.out = out;
  return launch(b, a, (hipStream_t)stream);
}

dqmc_status dqmc_debug_ratios(dqmc_batch* b, int32_t slice, double* out, void* stream) {
  if (!b || !out) return fail(DQMC_EINVAL, "batch/out is NULL");
  if (slice < 1 || slice > b->L) return fail(DQMC_EINVAL, "slice must be in [1, n_slices]");
  KArgs a = b->args;
  a.op = OP_DEBUG_RATIOS;
  a.slice = slice;
  a.out = out;
  return launch(b, a, (hipStream_t)stream);
}

dqmc_status dqmc_debug_propagators(dqmc_batch* b, double* out, void* stream) {
  if (!b || !out) return fail(DQMC_EINVAL, "batch/out is NULL");
  KArgs a = b->args;
  a.out = out;
  hipLaunchKernelGGL(copy_propagators_kernel, dim3(16), dim3(256), 0, (hipStream_t)stream, a);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_debug_phase_ticks(dqmc_batch* b, int64_t* out, void* stream) {
  if (!b || !out) return fail(DQMC_EINVAL, "batch/out is NULL");
  if (b->n_chains == 0) return DQMC_OK;
  hipLaunchKernelGGL(phase_ticks_kernel, dim3((b->n_chains + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, b->args, out);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_debug_philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                              uint64_t c3, int32_t n_blocks, uint64_t* out, void* stream) {
  if (!out || n_blocks < 0) return fail(DQMC_EINVAL, "bad philox arguments");
  if (n_blocks == 0) return DQMC_OK;
  hipLaunchKernelGGL(philox_kernel, dim3((n_blocks + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     k0, k1, c0, c1, c2, c3, n_blocks, out);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_debug_mfma(const double* a64, const double* b64, double* out64, const float* a32,
                            const float* b32, float* out32, void* stream) {
  if (!a64 || !b64 || !out64 || !a32 || !b32 || !out32) return fail(DQMC_EINVAL, "NULL argument");
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, a64, b64, out64,
                     a32, b32, out32);
  HIP_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status dqmc_graph_create(dqmc_graph** out, dqmc_batch* const* bs, const int32_t* n_sweeps,
                              int32_t n) {
  if (!out) return fail(DQMC_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || !bs || !n_sweeps) return fail(DQMC_EINVAL, "bad batch list");
  for (int i = 0; i < n; ++i)
    if (!bs[i] || n_sweeps[i] < 0) return fail(DQMC_EINVAL, "bad batch entry");
  dqmc_graph* g = new (std::nothrow) dqmc_graph;
  if (!g) return fail(DQMC_EDEVICE, "host allocation failed");
  g->args.resize(n);
  auto bail = [&](dqmc_status st) { delete g; return st; };
  hipError_t e = hipGraphCreate(&g->graph, 0);
  if (e != hipSuccess) return bail(fail(DQMC_EDEVICE, std::string("hipGraphCreate: ") + hipGetErrorString(e)));
  for (int i = 0; i < n; ++i) {
    if (n_sweeps[i] == 0 || bs[i]->n_chains == 0) continue;
    KArgs& a = g->args[i];
    a = bs[i]->args;
    a.op = OP_SWEEP;
    a.n_sweeps = n_sweeps[i];
    const KernelRef k = resolve(bs[i], OP_SWEEP);
    dqmc_status st = prepare(k);
    if (st != DQMC_OK) return bail(st);
    void* params[] = {&a};
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(k.fn);
    p.gridDim = dim3(bs[i]->n_chains);
    p.blockDim = dim3(NT);
    p.sharedMemBytes = (unsigned)k.lds;
    p.kernelParams = params;
    p.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, g->graph, nullptr, 0, &p);
    if (e != hipSuccess)
      return bail(fail(DQMC_EDEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e)));
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(fail(DQMC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)));
  *out = g;
  return DQMC_OK;
}

dqmc_status dqmc_graph_launch(dqmc_graph* g, void* stream) {
  if (!g) return fail(DQMC_EINVAL, "graph is NULL");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return DQMC_OK;
}

dqmc_status dqmc_graph_destroy(dqmc_graph* g) {
  delete g;
  return DQMC_OK;
}

dqmc_status dqmc_run_static(const dqmc_model* m, int32_t n_chains, const int8_t* fields,
                            const uint64_t* seeds, int32_t n_sweeps, dqmc_obs* obs, double* green,
                            int8_t* fields_out, void* stream) {
  if (!obs) return fail(DQMC_EINVAL, "obs is NULL");
  if (n_sweeps < 0) return fail(DQMC_EINVAL, "n_sweeps must be >= 0");
  Layout L;
  dqmc_status st = make_layout(m, n_chains, &L, true);
  if (st != DQMC_OK) return st;
  const size_t need = L.c_end + (size_t)n_chains * L.stride;
  if (need > DQMC_STATIC_BYTES) {
    std::snprintf(g_err, sizeof g_err,
                  "dqmc_run_static: %zu bytes of chain state exceed the static array (%zu bytes)",
                  need, (size_t)DQMC_STATIC_BYTES);
    return DQMC_EINVAL;
  }
  char* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != DQMC_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  dqmc_batch b;
  st = init_core(&b, L, m, n_chains, fields, seeds, ws, DQMC_STATIC_BYTES, s);
  if (st != DQMC_OK) return st;
  if (n_chains == 0) return DQMC_OK;
  if (n_sweeps > 0) {
    KArgs a = b.args;
    a.op = OP_SWEEP;
    a.n_sweeps = n_sweeps;
    st = launch(&b, a, s);
    if (st != DQMC_OK) return st;
  }
  hipLaunchKernelGGL(measure_kernel, dim3(n_chains), dim3(NT), 0, s, b.args, obs, green);
  HIP_TRY(hipGetLastError());
  if (fields_out) {
    hipLaunchKernelGGL(get_fields_kernel, dim3(n_chains), dim3(256), 0, s, b.args, fields_out);
    HIP_TRY(hipGetLastError());
  }
  // every chain's flags into the workspace's second error word, then to the host
  int* fw = (int*)(ws + L.c_err) + 1;
  hipLaunchKernelGGL(flags_or_kernel, dim3(1), dim3(NT), 0, s, (const dqmc_obs*)obs, n_chains, fw);
  HIP_TRY(hipGetLastError());
  int flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, fw, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flags) return fail(DQMC_ENUMERIC, "a chain raised a numerical flag");
  return DQMC_OK;
}

}  // extern "C"
