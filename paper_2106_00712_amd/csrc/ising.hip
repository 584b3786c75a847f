// Batched Metropolis sweeps of the square-lattice Ising model (main text eq. (1); one attempt
// per spin and sweep, supplement section I.3), many independent chains on one MI355X.
//
// One workgroup per chain; the L x L lattice (int8, at most 4 KiB) stays in LDS for the whole
// launch, so a sweep touches HBM only for the optional per-sweep series.  Thread t owns the four
// row-major sites 4t .. 4t+3 and the Philox4x64-10 block (t, 0, sweep, 2) whose four words are
// their acceptance uniforms; the checkerboard colours are two parallel steps separated by a
// workgroup barrier (a site only reads neighbours of the other colour).  The work is integer
// and ALU-bound: one Philox block per four attempts dominates.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "dqmc_error.hpp"
#include "ising.h"
#include "philox.hpp"

using namespace dqmc;

struct ising_batch {
  int L = 0, n_chains = 0, threads = 0;
  double J = 0, T = 0;
  double p[5] = {1, 1, 1, 1, 1};   // acceptance for k = s*h = -4, -2, 0, 2, 4
  int8_t* spins = nullptr;         // [n_chains][L*L]
  ising_obs* stats = nullptr;      // [n_chains]
  uint64_t* seeds = nullptr;       // [n_chains]
  int32_t* err = nullptr;          // init validation flag
};

namespace {

constexpr int MAX_L = 64;
constexpr int MAX_THREADS = MAX_L * MAX_L / 4;

#define ISING_TRY(expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(DQMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct IsingArgs {
  int L, n_sweeps, measure;
  double pm4, pm2, p0, pp2, pp4;   // acceptance for k = s*h = -4, -2, 0, 2, 4
  int8_t* spins;
  ising_obs* stats;
  const uint64_t* seeds;
  int32_t* series;
};

__device__ __forceinline__ int wave_sum_int(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__global__ __launch_bounds__(MAX_THREADS) void ising_init_kernel(int L, const int8_t* in,
                                                                 int8_t* spins, ising_obs* stats,
                                                                 const uint64_t* seeds, int32_t* err) {
  const int chain = blockIdx.x, n = L * L;
  const uint64_t seed = seeds[chain];
  int8_t* g = spins + (size_t)chain * n;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    int8_t v;
    if (in) {
      v = in[(size_t)chain * n + e];
      if (v != 1 && v != -1) atomicOr(err, 1);
    } else {
      const u64x4 w = philox4x64_10(u64x4{(uint64_t)(e >> 2), 0ull, 0ull, 0ull}, seed, 0ull);
      const uint64_t r = (e & 3) == 0 ? w.x0 : (e & 3) == 1 ? w.x1 : (e & 3) == 2 ? w.x2 : w.x3;
      v = (r & 1ull) ? 1 : -1;
    }
    g[e] = v;
  }
  if (threadIdx.x == 0) {
    ising_obs o = {};
    stats[chain] = o;
  }
}

__global__ __launch_bounds__(MAX_THREADS) void ising_sweep_kernel(IsingArgs a) {
  __shared__ int8_t S[MAX_L * MAX_L];
  __shared__ int red[3][MAX_THREADS / 64];
  const int chain = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int L = a.L, n = L * L, nblk = n >> 2;
  int8_t* g = a.spins + (size_t)chain * n;
  for (int e = tid; e < n; e += nt) S[e] = g[e];
  const uint64_t seed = a.seeds[chain];
  const int64_t sweep0 = a.stats[chain].sweeps_done;
  const bool act = tid < nblk;
  // the four sites of this thread, their colours and neighbours (right, left, down, up)
  int site[4], col[4], nr[4], nl[4], nd[4], nu[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int s = act ? 4 * tid + q : 0;
    const int x = s % L, y = s / L;
    site[q] = s;
    col[q] = (x + y) & 1;
    nr[q] = y * L + (x + 1 == L ? 0 : x + 1);
    nl[q] = y * L + (x == 0 ? L - 1 : x - 1);
    nd[q] = (y + 1 == L ? 0 : y + 1) * L + x;
    nu[q] = (y == 0 ? L - 1 : y - 1) * L + x;
  }
  __syncthreads();
  int64_t acc = 0, sam = 0, sm2 = 0, sb = 0, sb2 = 0;
  for (int k = 0; k < a.n_sweeps; ++k) {
    double u[4] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
      const u64x4 w = philox4x64_10(u64x4{(uint64_t)tid, 0ull, (uint64_t)(sweep0 + k), 2ull}, seed, 0ull);
      u[0] = unit53(w.x0);
      u[1] = unit53(w.x1);
      u[2] = unit53(w.x2);
      u[3] = unit53(w.x3);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (act) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (col[q] != c) continue;
          const int s = S[site[q]];
          const int h = S[nr[q]] + S[nl[q]] + S[nd[q]] + S[nu[q]];
          const int kk = s * h;
          const double p = kk == 4 ? a.pp4 : kk == 2 ? a.pp2 : kk == 0 ? a.p0 : kk == -2 ? a.pm2 : a.pm4;
          if (u[q] < p) {
            S[site[q]] = (int8_t)(-s);
            ++acc;
          }
        }
      }
      __syncthreads();
    }
    if (a.measure || a.series) {
      int m = 0, b = 0;
      if (act) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int s = S[site[q]];
          m += s;
          b += s * (S[nr[q]] + S[nd[q]]);
        }
      }
      m = wave_sum_int(m);
      b = wave_sum_int(b);
      if ((tid & 63) == 0) {
        red[0][tid >> 6] = m;
        red[1][tid >> 6] = b;
      }
      __syncthreads();
      if (tid == 0) {
        int M = 0, B = 0;
        for (int w = 0; w < nt / 64; ++w) {
          M += red[0][w];
          B += red[1][w];
        }
        if (a.measure) {
          sam += M < 0 ? -M : M;
          sm2 += (int64_t)M * M;
          sb += B;
          sb2 += (int64_t)B * B;
        }
        if (a.series) {
          int32_t* o = a.series + ((size_t)chain * a.n_sweeps + k) * 2;
          o[0] = M;
          o[1] = B;
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < n; e += nt) g[e] = S[e];
  const int at = wave_sum_int((int)acc);
  if ((tid & 63) == 0) red[2][tid >> 6] = at;
  __syncthreads();
  if (tid == 0) {
    int64_t A = 0;
    for (int w = 0; w < nt / 64; ++w) A += red[2][w];
    ising_obs o = a.stats[chain];
    o.sweeps_done += a.n_sweeps;
    o.accepted += A;
    if (a.measure) {
      o.n_meas += a.n_sweeps;
      o.sum_abs_m += sam;
      o.sum_m2 += sm2;
      o.sum_bond += sb;
      o.sum_bond2 += sb2;
    }
    a.stats[chain] = o;
  }
}

struct IsingLayout {
  size_t o_spins, o_stats, o_seeds, o_err, total;
};

IsingLayout ising_layout(int L, int n_chains) {
  IsingLayout l;
  size_t off = 0;
  l.o_spins = off;
  off += align256((size_t)n_chains * L * L);
  l.o_stats = off;
  off += align256((size_t)n_chains * sizeof(ising_obs));
  l.o_seeds = off;
  off += align256((size_t)n_chains * sizeof(uint64_t));
  l.o_err = off;
  off += 256;
  l.total = off;
  return l;
}

bool valid_size(int L) { return L >= 2 && L <= MAX_L && (L % 2) == 0; }

}  // namespace

extern "C" {

size_t ising_workspace_bytes(int32_t L, int32_t n_chains) {
  if (!valid_size(L) || n_chains < 0) return 0;
  return ising_layout(L, n_chains).total;
}

dqmc_status ising_init(ising_batch** out, int32_t L, double J, double T, int32_t n_chains,
                       const int8_t* spins, const uint64_t* seeds, void* workspace,
                       size_t ws_bytes, void* stream) {
  if (!out) return set_error(DQMC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_size(L)) return set_error(DQMC_EINVAL, "L must be even and in [2, 64]");
  if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(J))
    return set_error(DQMC_EINVAL, "need a finite T > 0 and a finite J");
  if (n_chains < 0) return set_error(DQMC_EINVAL, "n_chains must be >= 0");
  if (n_chains > 0 && (!seeds || !workspace)) return set_error(DQMC_EINVAL, "seeds/workspace is NULL");
  const IsingLayout l = ising_layout(L, n_chains);
  if (n_chains > 0 && ((uintptr_t)workspace & 255)) return set_error(DQMC_EINVAL, "workspace not 256-byte aligned");
  if (n_chains > 0 && ws_bytes < l.total) return set_error(DQMC_ENOMEM, "workspace too small");
  ising_batch* b = new (std::nothrow) ising_batch;
  if (!b) return set_error(DQMC_ENOMEM, "host allocation");
  b->L = L;
  b->n_chains = n_chains;
  b->J = J;
  b->T = T;
  for (int i = 0; i < 5; ++i) {
    const int kk = 2 * i - 4;
    const double dE = 2.0 * J * kk;
    b->p[i] = dE <= 0.0 ? 1.0 : std::exp(-dE / T);
  }
  b->threads = ((L * L / 4 + 63) / 64) * 64;
  char* ws = (char*)workspace;
  b->spins = (int8_t*)(ws + l.o_spins);
  b->stats = (ising_obs*)(ws + l.o_stats);
  b->seeds = (uint64_t*)(ws + l.o_seeds);
  b->err = (int32_t*)(ws + l.o_err);
  if (n_chains == 0) {
    *out = b;
    return DQMC_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  auto bail = [&](hipError_t e, const char* what) {
    delete b;
    return set_error(DQMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMemsetAsync(b->err, 0, sizeof(int32_t), s)) != hipSuccess) return bail(e, "memset");
  if ((e = hipMemcpyAsync(b->seeds, seeds, (size_t)n_chains * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return bail(e, "seed copy");
  hipLaunchKernelGGL(ising_init_kernel, dim3(n_chains), dim3(256), 0, s, L, spins, b->spins, b->stats,
                     b->seeds, b->err);
  if ((e = hipGetLastError()) != hipSuccess) return bail(e, "init launch");
  int32_t herr = 0;
  if ((e = hipMemcpyAsync(&herr, b->err, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return bail(e, "flag copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(e, "sync");
  if (herr) {
    delete b;
    return set_error(DQMC_EINVAL, "a spin value other than +-1");
  }
  *out = b;
  return DQMC_OK;
}

dqmc_status ising_sweep(ising_batch* b, int32_t n_sweeps, int32_t measure, int32_t* series,
                        void* stream) {
  if (!b) return set_error(DQMC_EINVAL, "batch is NULL");
  if (n_sweeps < 0) return set_error(DQMC_EINVAL, "n_sweeps must be >= 0");
  if (b->n_chains == 0 || n_sweeps == 0) return DQMC_OK;
  IsingArgs a;
  a.L = b->L;
  a.n_sweeps = n_sweeps;
  a.measure = measure ? 1 : 0;
  a.pm4 = b->p[0];
  a.pm2 = b->p[1];
  a.p0 = b->p[2];
  a.pp2 = b->p[3];
  a.pp4 = b->p[4];
  a.spins = b->spins;
  a.stats = b->stats;
  a.seeds = b->seeds;
  a.series = series;
  hipLaunchKernelGGL(ising_sweep_kernel, dim3(b->n_chains), dim3(b->threads), 0, (hipStream_t)stream, a);
  ISING_TRY(hipGetLastError());
  return DQMC_OK;
}

dqmc_status ising_stats(ising_batch* b, ising_obs* out, void* stream) {
  if (!b || !out) return set_error(DQMC_EINVAL, "batch/out is NULL");
  if (b->n_chains == 0) return DQMC_OK;
  ISING_TRY(hipMemcpyAsync(out, b->stats, (size_t)b->n_chains * sizeof(ising_obs),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return DQMC_OK;
}

dqmc_status ising_get_spins(ising_batch* b, int8_t* out, void* stream) {
  if (!b || !out) return set_error(DQMC_EINVAL, "batch/out is NULL");
  if (b->n_chains == 0) return DQMC_OK;
  ISING_TRY(hipMemcpyAsync(out, b->spins, (size_t)b->n_chains * b->L * b->L, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  return DQMC_OK;
}

dqmc_status ising_destroy(ising_batch* b) {
  delete b;
  return DQMC_OK;
}

}  // extern "C"
