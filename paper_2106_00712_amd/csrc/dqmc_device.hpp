// Device side of the batched DQMC sweep (gfx950 / CDNA4).
//
// One workgroup of 256 threads (4 wave64s) owns one Markov chain for the whole call: the
// kernels are persistent over slices and sweeps, and all per-chain state is resident either in
// LDS (Green's functions and two work matrices, "small" variant) or in the chain's slice of the
// caller's workspace ("large" variant).  Dense products run on the matrix cores through
// 16x16x4 MFMA tiles (FP64, or FP32 for the wraps and delayed updates in FP32-wrap precision);
// the latency-bound parts (the sequential Metropolis loop, pivot searches) use wave-synchronous
// LDS traffic and wavefront reductions.
//
// Notation of the paper's supplement, section I.2: L slices of width dtau, HS field s_{i,l}=+-1,
// cosh(nu) = e^{U dtau/2}, B^sigma_l = e^{sigma nu Diag(s_l)} e^{-dtau T}, weight
// prod_sigma det(I + B^sigma(L,0)).  Everything beyond that (Green's function, wrap, ratio,
// Sherman-Morrison/submatrix updates, UDT stabilisation) is derived in the comments below.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

// Pointer into LDS (address space 3), for arguments of functions that are not inlined and for
// LDS areas reached through generic pointers.
#ifndef DQMC_LDS
#define DQMC_LDS __attribute__((address_space(3)))
#endif
// Pointer into global memory (address space 1): loads through it are global loads, counted by
// vmcnt alone, where loads through generic pointers are flat loads that also hold lgkmcnt (so a
// wait for LDS reads would wait for them too).
#ifndef DQMC_GLB
#define DQMC_GLB __attribute__((address_space(1)))
#endif

namespace dqmc {

constexpr int NT = 256;        // threads per workgroup (one chain)
constexpr int NW = NT / 64;    // wavefronts per workgroup

enum { OP_INIT = 0, OP_SWEEP = 1, OP_DEBUG_GREEN = 2, OP_DEBUG_RATIOS = 3 };
enum { FLAG_NONFINITE = 1, FLAG_NEGATIVE = 2, FLAG_DRIFT = 4, FLAG_SINGULAR = 8 };

// Per-chain bookkeeping kept in the workspace.
struct ChainStats {
  uint64_t seed;
  int64_t sweeps_done, attempted, accepted, near_ties;
  double max_drift, max_logdet_err;
  double logdet[2];
  int32_t flags, pad;
  int64_t ticks[16];  // wall-clock ticks (100 MHz) spent per phase, see enum Phase
  double slice_docc, slice_kin;   // sums of the per-slice equal-time estimators
  int64_t slice_meas;
  int32_t stack_ok;   // the right UDT stack describes the current fields (alternating sweeps)
  int32_t pad2;
};

// Phases of a sweep timed by thread 0 between workgroup barriers.
enum Phase { PH_RIGHT = 0, PH_WRAP = 1, PH_DECIDE = 2, PH_PANEL = 3, PH_FLUSH = 4, PH_LEFT = 5,
             PH_FRESH = 6, PH_SWEEP = 7,
             // finer split of the stabilisation work (fast path)
             PH_CHUNK = 8, PH_QR = 9, PH_QFORM = 10, PH_TMUL = 11, PH_FGEMM = 12, PH_GJ = 13,
             PH_GOUT = 14, PH_PARK = 15 };
struct PhaseClock {
  int64_t t;
  __device__ __forceinline__ void start() { if (threadIdx.x == 0) t = wall_clock64(); }
  __device__ __forceinline__ void stop(ChainStats* st, int ph) {
    if (threadIdx.x == 0) { int64_t e = wall_clock64(); st->ticks[ph] += e - t; t = e; }
  }
};

// Everything a kernel launch needs (passed by value).
struct KArgs {
  int n, np, L, stab, J, K, n_chains, op, slice, n_wraps, n_sweeps, gen_fields;
  int KT;               // accumulated delayed-update rank of the N > 64 workspace kernels (0: none)
  int sweep_mode;       // bit 0: alternating up/down sweeps, bit 1: per-slice measurements
  double nu, drift_limit;
  double ev[2];     // e^{+nu}, e^{-nu}
  double dup[2];    // Delta^up(s)   = e^{-2 nu s} - 1 for s = -1 (index 0), s = +1 (index 1)
  double ddn[2];    // Delta^down(s) = e^{+2 nu s} - 1
  const double* expK;
  const double* expKinv;
  const float* expK32;
  const float* expKinv32;
  const double* Tm;     // hopping (np x np, zero padded), for the kinetic energy
  const double* eye;    // n x n identity zero-padded to np x np
  const double* ones;   // np ones
  int* err;             // device error word (field validation)
  const int8_t* fields_in;
  const uint64_t* seeds;
  const int32_t* slots;   // init over a subset: block b initialises chain slots[b] from input b
  const int32_t* counts;  // per-chain sweeps of this launch (NULL: n_sweeps for every chain)
  char* base;
  size_t stride;        // bytes per chain
  size_t o_fields, o_G64, o_Gw, o_stack, o_left, o_work, o_xy, o_stats;
  size_t o_qrv;         // scratch of the blocked factorisations (0: unblocked only)
  size_t o_lstack;      // left UDT stack of the alternating sweeps (0: none)
  int qr_blocked;       // stabilisation QR: 1 blocked with pre-sorted columns, 0 column-pivoted
  double* out;
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct acc4;
template <> struct acc4<double> { typedef d4 type; };
template <> struct acc4<float> { typedef f4 type; };

// acc += A(16x4) B(4x16); lane l supplies A[l%16][l/16] and B[l/16][l%16].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of output register v held by lane l (column = l % 16).  The FP64 instruction returns four
// row groups of one row each (rows v*4 + l/16); the FP32 one a single group of four rows
// (rows 4*(l/16) + v).  Checked on the device by dqmc_debug_mfma.
template <typename T> __device__ __forceinline__ int out_row(int v, int lane);
template <> __device__ __forceinline__ int out_row<double>(int v, int lane) { return 4 * v + (lane >> 4); }
template <> __device__ __forceinline__ int out_row<float>(int v, int lane) { return 4 * (lane >> 4) + v; }

// Compiler and LDS ordering point for wave-synchronous code (one wave, no s_barrier).
__device__ __forceinline__ void wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// --------------------------------------------------------------------------------- GEMM tiles
// nb independent products C_b(i,j) = sum_{k<K} A_b(i,k) B_b(k,j), i < M, j < Nc (multiples of
// 16), K a multiple of 4; A_b(i,k) = A_b[i*sai + k*sak], B_b(k,j) = B_b[k*sbk + j*sbj].
// The 16x16 output tiles of all nb products are dealt round-robin to the four wavefronts;
// epi(b, i, j, value) is called exactly once per output element, by the lane owning it.
template <typename T, typename Epi>
__device__ __forceinline__ void wg_gemm(int nb, int M, int Nc, int K, const T* A0, const T* A1,
                                        int sai, int sak, const T* B0, const T* B1, int sbk,
                                        int sbj, Epi epi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tn = Nc >> 4, tpb = (M >> 4) * tn;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < nb * tpb; t += NW) {
    const int b = t / tpb, tt = t - b * tpb;
    const int ti = tt / tn, tj = tt - ti * tn;
    const T* a = (b ? A1 : A0) + (ti * 16 + li) * sai + lk * sak;
    const T* bb = (b ? B1 : B0) + lk * sbk + (tj * 16 + li) * sbj;
    typename acc4<T>::type acc = {0, 0, 0, 0};
    int k = 0;
    for (; k + 16 <= K; k += 16) {
      T a0 = a[(k + 0) * sak], a1 = a[(k + 4) * sak], a2 = a[(k + 8) * sak], a3 = a[(k + 12) * sak];
      T b0 = bb[(k + 0) * sbk], b1 = bb[(k + 4) * sbk], b2 = bb[(k + 8) * sbk], b3 = bb[(k + 12) * sbk];
      acc = mfma(a0, b0, acc);
      acc = mfma(a1, b1, acc);
      acc = mfma(a2, b2, acc);
      acc = mfma(a3, b3, acc);
    }
    for (; k < K; k += 4) acc = mfma(a[k * sak], bb[k * sbk], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) epi(b, ti * 16 + out_row<T>(v, lane), tj * 16 + li, acc[v]);
  }
}

// ------------------------------------------------------------------------------ workspace products
// LDS scratch of the workspace kernels' blocked factorisations (partial sums, the current panel's
// T and pivot block), in doubles; it also sizes their LDS layout on the host.
constexpr int TG_STAGE_DOUBLES = 4096;

// Matrix products of the workspace kernels (N > 64, matrices in the chain's workspace):
// C_b(i, j) = sum_{k < K} A_b(i, k) B_b(k, j) for b < nb, i < M, j < Nc, with
// A_b(i, k) = A_b[i sai + k sak] and B_b(k, j) = B_b[k sbk + j sbj].  Each wavefront computes
// whole 32 x 32 output tiles (2 x 2 MFMA tiles) on its own, reading its operands straight from
// global memory with WK_U k-steps of 4 in flight per lane: no LDS staging and no workgroup
// barrier, so the four wavefronts' loads overlap each other's matrix-core work.  (An LDS-staged
// 64 x 64 macro-tile shared by the workgroup measured slower at these sizes: it waits on memory
// once per 16-deep panel for the whole workgroup.)  The k order is steps of 4 ascending, as in
// wg_gemm.  Contract: operands in global memory (the workspace or the model constants), never
// LDS; M and Nc multiples of 16; K a multiple of 4; epi(b, i, j, value) is called once per
// output element by the lane that owns it; no barrier inside (callers order the calls).
// ADD: C_b[i ldc + j] += (A_b B_b)(i, j) instead of epi, with the tile of C loaded together with
// the first operands (no memory round trip after the products).
constexpr int WK_U = 8;
template <typename T, bool ADD, typename Epi>
__device__ __forceinline__ void wave_gemm_impl(int nb, int M, int Nc, int K, const T* A0g, const T* A1g,
                                               int sai, int sak, const T* B0g, const T* B1g, int sbk,
                                               int sbj, T* C0g, T* C1g, int ldc, Epi epi) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (M + 31) >> 5, nt = (Nc + 31) >> 5;
  const DQMC_GLB T* A0 = (const DQMC_GLB T*)A0g;
  const DQMC_GLB T* A1 = (const DQMC_GLB T*)A1g;
  const DQMC_GLB T* B0 = (const DQMC_GLB T*)B0g;
  const DQMC_GLB T* B1 = (const DQMC_GLB T*)B1g;
  for (int t = wave; t < nb * mt * nt; t += NW) {
    const int b = t / (mt * nt), tt = t - b * (mt * nt);
    const int i0 = (tt / nt) * 32, j0 = (tt - (tt / nt) * nt) * 32;
    const DQMC_GLB T* A = b ? A1 : A0;
    const DQMC_GLB T* B = b ? B1 : B0;
    const int ia = i0 + li, ib = i0 + 16 + li, ja = j0 + li, jb = j0 + 16 + li;
    const bool va = ia < M, vb = ib < M, wa = ja < Nc, wb = jb < Nc;
    typename acc4<T>::type acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[r][q] = typename acc4<T>::type{0, 0, 0, 0};
    DQMC_GLB T* C = (DQMC_GLB T*)(b ? C1g : C0g);
    T cp[2][2][4];
    if (ADD) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool live = (i0 + 16 * r < M) && (j0 + 16 * q < Nc);
            cp[r][q][v] = live ? C[(size_t)(i0 + 16 * r + out_row<T>(v, lane)) * ldc + j0 + 16 * q + li] : (T)0;
          }
    }
    for (int k0 = 0; k0 < K; k0 += 4 * WK_U) {
      T a[WK_U][2], bv[WK_U][2];
#pragma unroll
      for (int s2 = 0; s2 < WK_U; ++s2) {
        const int k = k0 + 4 * s2 + lk;
        const bool kv = k < K;
        a[s2][0] = (kv && va) ? A[(size_t)ia * sai + (size_t)k * sak] : (T)0;
        a[s2][1] = (kv && vb) ? A[(size_t)ib * sai + (size_t)k * sak] : (T)0;
        bv[s2][0] = (kv && wa) ? B[(size_t)k * sbk + (size_t)ja * sbj] : (T)0;
        bv[s2][1] = (kv && wb) ? B[(size_t)k * sbk + (size_t)jb * sbj] : (T)0;
      }
#pragma unroll
      for (int s2 = 0; s2 < WK_U; ++s2) {
        if (k0 + 4 * s2 < K) {
          acc[0][0] = mfma(a[s2][0], bv[s2][0], acc[0][0]);
          if (wb) acc[0][1] = mfma(a[s2][0], bv[s2][1], acc[0][1]);
          if (vb) acc[1][0] = mfma(a[s2][1], bv[s2][0], acc[1][0]);
          if (vb && wb) acc[1][1] = mfma(a[s2][1], bv[s2][1], acc[1][1]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (i0 + 16 * r >= M || j0 + 16 * q >= Nc) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * r + out_row<T>(v, lane), j = j0 + 16 * q + li;
          if (ADD) C[(size_t)i * ldc + j] = cp[r][q][v] + acc[r][q][v];
          else epi(b, i, j, acc[r][q][v]);
        }
      }
  }
}
template <typename T, typename Epi>
__device__ __forceinline__ void wave_gemm(int nb, int M, int Nc, int K, const T* A0, const T* A1,
                                          int sai, int sak, const T* B0, const T* B1, int sbk,
                                          int sbj, Epi epi) {
  wave_gemm_impl<T, false>(nb, M, Nc, K, A0, A1, sai, sak, B0, B1, sbk, sbj, (T*)nullptr, (T*)nullptr,
                           0, epi);
}
// C_b += A_b B_b (C_b row-major with leading dimension ldc, in global memory).
template <typename T>
__device__ __forceinline__ void wave_gemm_add(int nb, int M, int Nc, int K, const T* A0, const T* A1,
                                              int sai, int sak, const T* B0, const T* B1, int sbk,
                                              int sbj, T* C0, T* C1, int ldc) {
  wave_gemm_impl<T, true>(nb, M, Nc, K, A0, A1, sai, sak, B0, B1, sbk, sbj, C0, C1, ldc,
                          [](int, int, int, T) {});
}

// ------------------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}
// Sum over the 4 consecutive lanes of a column group.
__device__ __forceinline__ double group4_sum(double x) {
  x += __shfl_xor(x, 1);
  x += __shfl_xor(x, 2);
  return x;
}

// LDS scratch the reductions use: red[2][NW] doubles and redi[2][NW] ints, double-buffered by
// the parity of the call so that one barrier per reduction suffices.
struct Red {
  double* v;
  int* i;
  int parity;
};

// Largest value over the workgroup (every thread contributes x); returns it to all threads.
__device__ __forceinline__ double wg_max(double x, Red& r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_max(x);
  double* buf = r.v + r.parity * NW;
  r.parity ^= 1;
  if (lane == 0) buf[wave] = x;
  __syncthreads();
  double m = buf[0];
  for (int w = 1; w < NW; ++w) m = fmax(m, buf[w]);
  return m;
}

// Index of the largest key over the workgroup (ties -> smallest index); every thread offers
// one (key, idx) pair, idx < 0 meaning "no candidate".  Returns the winner to all threads.
__device__ __forceinline__ int wg_argmax(double key, int idx, Red& r) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (idx < 0) key = -1.0;
  for (int o = 32; o > 0; o >>= 1) {
    double k2 = __shfl_xor(key, o);
    int i2 = __shfl_xor(idx, o);
    bool take = (i2 >= 0) && (idx < 0 || k2 > key || (k2 == key && i2 < idx));
    if (take) { key = k2; idx = i2; }
  }
  double* bv = r.v + r.parity * NW;
  int* bi = r.i + r.parity * NW;
  r.parity ^= 1;
  if (lane == 0) { bv[wave] = key; bi[wave] = idx; }
  __syncthreads();
  double bk = bv[0];
  int best = bi[0];
  for (int w = 1; w < NW; ++w) {
    double k2 = bv[w];
    int i2 = bi[w];
    if (i2 >= 0 && (best < 0 || k2 > bk || (k2 == bk && i2 < best))) { bk = k2; best = i2; }
  }
  return best;
}

// Philox4x64-10: philox.hpp
// Acceptance uniform of (global sweep, 0-based slice, site): counter (site, slice, sweep, 1),
// key (seed, 0), first word, top 53 bits.
__device__ __forceinline__ double accept_uniform(uint64_t seed, int64_t sweep, int slice, int site) {
  u64x4 w = philox4x64_10(u64x4{(uint64_t)site, (uint64_t)slice, (uint64_t)sweep, 1ull}, seed, 0ull);
  return (double)(w.x0 >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------------------------ chain context
template <typename WT>
struct Ctx {
  const KArgs* a;
  int n, np, L, stab, J, K;
  ChainStats* st;
  int8_t* f;          // fields [L][np]
  double* G64;        // [2][np*np] fresh G(0) record
  WT* G[2];           // working Green's functions (LDS or global)
  double* w1;         // work matrices (LDS or global), np*np doubles each
  double* w2;
  WT* xy;             // delayed-update panels: X_up, Y_up, X_dn, Y_dn (np*K each)
  double* stack;      // right UDT stack [2][J][U, T, d]
  double* left;       // left UDT [2][U, T0, T1, d]
  double* qrv;        // blocked QR: reflectors V (np x np, column-major) then T factors, or NULL
  double* lstack;     // left UDT stack [2][J][U, T, d] of the alternating sweeps, or NULL
  // LDS vectors
  double *vd, *bt, *nrm, *dtmp, *sr, *sc;   // sr/sc: [2][np] row/column scale factors
  int* ordv;          // [np] pivot order / used marks
  int* rank;          // [np]
  double *gb, *xb, *yb;   // [2][K*K] each
  double *cfu, *cfd, *ublk;  // [K]
  int *site, *sblk, *cnt;   // [K], [K], [4]
  double* misc;       // [16]
  double* stage;      // LDS staging of the tiled products (matrices in the workspace), else NULL
  Red red;
};

template <typename WT>
__device__ __forceinline__ const WT* kexp(const KArgs& a);
template <> __device__ __forceinline__ const double* kexp<double>(const KArgs& a) { return a.expK; }
template <> __device__ __forceinline__ const float* kexp<float>(const KArgs& a) { return a.expK32; }
template <typename WT>
__device__ __forceinline__ const WT* kexpinv(const KArgs& a);
template <> __device__ __forceinline__ const double* kexpinv<double>(const KArgs& a) { return a.expKinv; }
template <> __device__ __forceinline__ const float* kexpinv<float>(const KArgs& a) { return a.expKinv32; }

// Bytes of LDS the vector area needs (both variants) and the matrix area (small variant).
__host__ __device__ inline size_t lds_vec_doubles(int np, int K) {
  return 2 * NW + NW + 6 * (size_t)np + 4 * (size_t)np + 6 * (size_t)K * K + 3 * (size_t)K +
         (3 * (size_t)K + 8) / 2 + 1 + 16 + (2 * (size_t)np + 1) / 2 + 8;
}
template <typename WT>
__host__ __device__ inline size_t lds_mat_bytes(int np) {
  return 2 * (size_t)np * np * sizeof(WT) + 2 * (size_t)np * np * sizeof(double);
}

template <typename WT, bool SMALL>
__device__ inline Ctx<WT> make_ctx(const KArgs& a, int chain, double* lds) {
  Ctx<WT> c;
  c.a = &a;
  c.n = a.n; c.np = a.np; c.L = a.L; c.stab = a.stab; c.J = a.J; c.K = a.K;
  const int np = a.np, K = a.K;
  const size_t nn = (size_t)np * np;
  char* cb = a.base + (size_t)chain * a.stride;
  c.st = (ChainStats*)(cb + a.o_stats);
  c.f = (int8_t*)(cb + a.o_fields);
  c.G64 = (double*)(cb + a.o_G64);
  c.stack = (double*)(cb + a.o_stack);
  c.left = (double*)(cb + a.o_left);
  c.qrv = a.o_qrv ? (double*)(cb + a.o_qrv) : nullptr;
  c.lstack = a.o_lstack ? (double*)(cb + a.o_lstack) : nullptr;
  double* p = lds;
  if (SMALL) {
    WT* g = (WT*)p;
    c.G[0] = g;
    c.G[1] = g + nn;
    p = (double*)(g + 2 * nn);
    c.w1 = p;
    c.w2 = p + nn;
    p += 2 * nn;
    c.xy = (WT*)c.w1;   // the panels reuse the work matrices during the Metropolis loop
  } else {
    WT* g = (WT*)(cb + a.o_Gw);
    c.G[0] = g;
    c.G[1] = g + nn;
    c.w1 = (double*)(cb + a.o_work);
    c.w2 = c.w1 + nn;
    c.xy = (WT*)(cb + a.o_xy);
  }
  c.stage = nullptr;
  if (!SMALL) {
    c.stage = p;
    p += TG_STAGE_DOUBLES;
  }
  c.red.v = p; p += 2 * NW;
  c.misc = p; p += 16;
  c.vd = p; p += np;
  c.bt = p; p += np;
  c.nrm = p; p += np;
  c.dtmp = p; p += np;
  c.sr = p; p += 2 * np;
  c.sc = p; p += 2 * np;
  c.gb = p; p += 2 * (size_t)K * K;
  c.xb = p; p += 2 * (size_t)K * K;
  c.yb = p; p += 2 * (size_t)K * K;
  c.cfu = p; p += K;
  c.cfd = p; p += K;
  c.ublk = p; p += K;
  int* ip = (int*)p;
  c.red.i = ip; ip += 2 * NW;
  c.site = ip; ip += K;
  c.sblk = ip; ip += K;
  c.cnt = ip; ip += 4;
  c.ordv = ip; ip += np;
  c.rank = ip; ip += np;
  c.red.parity = 0;
  return c;
}

// Products of the generic path: tiled through the LDS staging area when the matrices live in the
// workspace, straight from LDS otherwise.
template <typename T, typename WT, typename Epi>
__device__ __forceinline__ void ctx_gemm(Ctx<WT>& c, int nb, int M, int Nc, int K, const T* A0,
                                         const T* A1, int sai, int sak, const T* B0, const T* B1,
                                         int sbk, int sbj, Epi epi) {
  if (c.stage) wave_gemm<T>(nb, M, Nc, K, A0, A1, sai, sak, B0, B1, sbk, sbj, epi);
  else wg_gemm<T>(nb, M, Nc, K, A0, A1, sai, sak, B0, B1, sbk, sbj, epi);
}

// ------------------------------------------------------------------------------ helpers
// e^{sigma nu s} for s = +-1 (sigma = +1 for spin index 0, -1 for 1).
__device__ __forceinline__ double vfac(const KArgs& a, int spin, int s) {
  return ((s > 0) == (spin == 0)) ? a.ev[0] : a.ev[1];
}

// dst = U Diag(d) (n x n in np x np, zero padded), optionally with rows scaled by rs[].
__device__ inline void form_ud(int np, const double* U, const double* d, const double* rs, double* dst) {
  for (int e = threadIdx.x; e < np * np; e += NT) {
    int i = e / np, j = e - i * np;
    double v = U[e] * d[j];
    if (rs) v *= rs[i];
    dst[e] = v;
  }
}

// Fill the row-scale vector sr[spin][i] = e^{sigma nu s_{l,i}} (1 on padding) for slice index
// li (0-based) of the field, both spins, and its inverse into sc.
template <typename WT>
__device__ inline void slice_scales(Ctx<WT>& c, int li) {
  const KArgs& a = *c.a;
  for (int e = threadIdx.x; e < 2 * c.np; e += NT) {
    int sp = e / c.np, i = e - sp * c.np;
    double v = 1.0, w = 1.0;
    if (i < c.n) {
      int s = c.f[(size_t)li * c.np + i];
      v = vfac(a, sp, s);
      w = vfac(a, sp, -s);
    }
    c.sr[e] = v;
    c.sc[e] = w;
  }
}

// ------------------------------------------------------------------------------ QR / UDT
// Sum over the 64 lanes by DPP (row_shr 1, 2, 4, 8 inclusive scans within each 16-lane row,
// then row_bcast:15 and row_bcast:31 carry the row totals up; lane 63 holds the sum).
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x += dpp_d<0x111>(x);
  x += dpp_d<0x112>(x);
  x += dpp_d<0x114>(x);
  x += dpp_d<0x118>(x);
  x += dpp_d<0x142, 0xa>(x);
  x += dpp_d<0x143, 0xc>(x);
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
  return __hiloint2double(hi, lo);
}

// Column-pivoted Householder QR (Golub & Van Loan, Alg. 5.4.1) of the n x n leading block of
// X stored column-major (element (r, col) at X[col * np + r]), with implicit pivoting: columns
// stay in place, ordv[j] is the column chosen at step j, rank[col] the step at which column col
// was chosen.  On return row j of column ordv[j'] (j <= j') holds R[j][j']; column ordv[j] below
// row j holds the Householder vector v_j (v_j[j] in vd[j]) and bt[j] = beta_j = 2 / (v_j^T v_j).
// Pivot = the remaining column of largest norm over the remaining rows, recomputed exactly at
// every step.  One wavefront per column: every access runs down a contiguous column.
template <typename WT>
__device__ __forceinline__ void wg_qrp(Ctx<WT>& c, double* X) {
  const int n = c.n, np = c.np, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* vb = c.sc;   // the pivot column of the current step (LDS)
  for (int k = tid; k < n; k += NT) c.rank[k] = -1;
  for (int col = wave; col < n; col += NW) {
    double s = 0;
    for (int r = lane; r < n; r += 64) { const double x = X[(size_t)col * np + r]; s += x * x; }
    s = wave_sum_dpp(s);
    if (lane == 0) c.nrm[col] = s;
  }
  double alpha_prev = 0, v0_prev = 0, beta_prev = 0;
  int p_prev = -1;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // publish the previous step's R diagonal and reflector (column p_prev is no longer read)
    if (tid == 0 && p_prev >= 0) {
      X[(size_t)p_prev * np + (j - 1)] = alpha_prev;
      c.vd[j - 1] = v0_prev;
      c.bt[j - 1] = beta_prev;
    }
    double key = -1.0;
    int idx = -1;
    for (int k = tid; k < n; k += NT) {
      if (c.rank[k] < 0) {
        const double v = c.nrm[k];
        if (idx < 0 || v > key) { key = v; idx = k; }
      }
    }
    const int p = wg_argmax(key, idx, c.red);
    const double* xp = X + (size_t)p * np;
    const double xj = xp[j];
    const double nx = sqrt(c.nrm[p]);
    const double alpha = (xj >= 0.0) ? -nx : nx;
    const double beta = (nx > 0.0) ? 1.0 / (alpha * (alpha - xj)) : 0.0;
    const double v0 = xj - alpha;
    for (int r = j + tid; r < n; r += NT) vb[r] = (r == j) ? v0 : xp[r];
    if (tid == 0) { c.rank[p] = j; c.ordv[j] = p; }
    __syncthreads();
    // apply H_j = I - beta v v^T to every remaining column, recomputing its norm below row j
    for (int col = wave; col < n; col += NW) {
      if (col == p || c.rank[col] >= 0) continue;
      double* xc = X + (size_t)col * np;
      double w = 0;
      for (int r = j + lane; r < n; r += 64) w += vb[r] * xc[r];
      w = wave_sum_dpp(w) * beta;
      double s2 = 0;
      for (int r = j + lane; r < n; r += 64) {
        const double x = xc[r] - w * vb[r];
        xc[r] = x;
        if (r > j) s2 += x * x;
      }
      s2 = wave_sum_dpp(s2);
      if (lane == 0) c.nrm[col] = s2;
    }
    alpha_prev = alpha; v0_prev = v0; beta_prev = beta; p_prev = p;
    __syncthreads();
  }
  if (tid == 0 && p_prev >= 0) {
    X[(size_t)p_prev * np + (n - 1)] = alpha_prev;
    c.vd[n - 1] = v0_prev;
    c.bt[n - 1] = beta_prev;
  }
  __syncthreads();
}

// wg_qrp for matrices in the workspace (np <= 64 CR): the same steps, pivots and per-lane
// summation order (so the same bits), with each column's active part held in registers between
// its dot product and its update instead of being read twice, and QC columns per wavefront in
// flight so that their memory latencies overlap.  X is read and written as global memory (the
// waits for the LDS vectors then do not wait for it).  vb: the pivot column (LDS, np doubles).
constexpr int QC = 8;   // columns per wavefront per step of the trailing update
template <int CR>
__device__ __noinline__ void qrp_columns(int n, int np, double* Xg, DQMC_LDS double* nrm,
                                         DQMC_LDS int* rank, DQMC_LDS int* ordv, DQMC_LDS double* vb,
                                         DQMC_LDS double* vd, DQMC_LDS double* bt,
                                         DQMC_LDS double* redv, DQMC_LDS int* redi) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  DQMC_GLB double* X = (DQMC_GLB double*)Xg;
  for (int k = tid; k < n; k += NT) rank[k] = -1;
  for (int col = wave; col < n; col += NW) {
    double s = 0;
    for (int r = lane; r < n; r += 64) { const double x = X[(size_t)col * np + r]; s += x * x; }
    s = wave_sum_dpp(s);
    if (lane == 0) nrm[col] = s;
  }
  double alpha_prev = 0, v0_prev = 0, beta_prev = 0;
  int p_prev = -1;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0 && p_prev >= 0) {
      X[(size_t)p_prev * np + (j - 1)] = alpha_prev;
      vd[j - 1] = v0_prev;
      bt[j - 1] = beta_prev;
    }
    // pivot: the remaining column of largest norm, ties to the lower index
    double key = -1.0;
    int idx = -1;
    for (int k = tid; k < n; k += NT) {
      if (rank[k] < 0) {
        const double v = nrm[k];
        if (idx < 0 || v > key) { key = v; idx = k; }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double k2 = __shfl_xor(key, o);
      const int i2 = __shfl_xor(idx, o);
      if (i2 >= 0 && (idx < 0 || k2 > key || (k2 == key && i2 < idx))) { key = k2; idx = i2; }
    }
    if (lane == 0) { redv[wave] = key; redi[wave] = idx; }
    __syncthreads();
    int p = redi[0];
    {
      double bk = redv[0];
      for (int w = 1; w < NW; ++w) {
        const double k2 = redv[w];
        const int i2 = redi[w];
        if (i2 >= 0 && (p < 0 || k2 > bk || (k2 == bk && i2 < p))) { bk = k2; p = i2; }
      }
    }
    p = (p >= 0 && p < n) ? p : j;
    const DQMC_GLB double* xp = X + (size_t)p * np;
    const double xj = xp[j];
    const double nx = sqrt(nrm[p]);
    const double alpha = (xj >= 0.0) ? -nx : nx;
    const double beta = (nx > 0.0) ? 1.0 / (alpha * (alpha - xj)) : 0.0;
    const double v0 = xj - alpha;
    for (int r = j + tid; r < n; r += NT) vb[r] = (r == j) ? v0 : xp[r];
    if (tid == 0) { rank[p] = j; ordv[j] = p; }
    __syncthreads();
    // trailing columns col0 + q NW (q < QC) of this wavefront: y = x - beta (v^T x) v
    for (int col0 = wave; col0 < n; col0 += QC * NW) {
      bool use[QC];
      bool any = false;
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        const int cq = col0 + q * NW;
        use[q] = (cq < n) && (cq != p) && rank[cq] < 0;
        any = any || use[q];
      }
      if (!any) continue;
      DQMC_GLB double* xq[QC];
#pragma unroll
      for (int q = 0; q < QC; ++q) xq[q] = X + (size_t)(use[q] ? col0 + q * NW : col0) * np;
      double rq[QC][CR];
#pragma unroll
      for (int t = 0; t < CR; ++t) {
        const int r = j + lane + 64 * t;
#pragma unroll
        for (int q = 0; q < QC; ++q) rq[q][t] = (use[q] && r < n) ? xq[q][r] : 0.0;
      }
      double w[QC];
#pragma unroll
      for (int q = 0; q < QC; ++q) w[q] = 0.0;
#pragma unroll
      for (int t = 0; t < CR; ++t) {
        const int r = j + lane + 64 * t;
        if (r < n) {
#pragma unroll
          for (int q = 0; q < QC; ++q) w[q] += vb[r] * rq[q][t];
        }
      }
#pragma unroll
      for (int q = 0; q < QC; ++q)
        if (use[q]) w[q] = wave_sum_dpp(w[q]) * beta;
      double sq[QC];
#pragma unroll
      for (int q = 0; q < QC; ++q) sq[q] = 0.0;
#pragma unroll
      for (int t = 0; t < CR; ++t) {
        const int r = j + lane + 64 * t;
        if (r < n) {
          const double v = vb[r];
#pragma unroll
          for (int q = 0; q < QC; ++q) {
            const double y = rq[q][t] - w[q] * v;
            if (use[q]) xq[q][r] = y;
            if (r > j) sq[q] += y * y;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < QC; ++q)
        if (use[q]) {
          const double sn = wave_sum_dpp(sq[q]);
          if (lane == 0) nrm[col0 + q * NW] = sn;
        }
    }
    alpha_prev = alpha; v0_prev = v0; beta_prev = beta; p_prev = p;
    __syncthreads();
  }
  if (tid == 0 && p_prev >= 0) {
    X[(size_t)p_prev * np + (n - 1)] = alpha_prev;
    vd[n - 1] = v0_prev;
    bt[n - 1] = beta_prev;
  }
  __syncthreads();
}

// Column jj of Q = H_0 H_1 ... H_jj e_jj (later reflectors do not touch e_jj), one wavefront per
// column with the column in registers (element r = lane + 64 t), written to Ud (row-major).
template <int CR>
__device__ __forceinline__ void q_columns(int n, int np, const double* X, const double* vd,
                                          const double* bt, const int* ordv, double* Ud) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jj = wave; jj < np; jj += NW) {
    double q[CR];
#pragma unroll
    for (int t = 0; t < CR; ++t) q[t] = (lane + 64 * t == jj && jj < n) ? 1.0 : 0.0;
    if (jj < n) {
      for (int j = jj; j >= 0; --j) {
        const double* v = X + (size_t)ordv[j] * np;
        const double v0 = vd[j];
        double w = 0;
#pragma unroll
        for (int t = 0; t < CR; ++t) {
          const int r = lane + 64 * t;
          if (r >= j && r < n) w += (r == j ? v0 : v[r]) * q[t];
        }
        w = wave_sum_dpp(w) * bt[j];
#pragma unroll
        for (int t = 0; t < CR; ++t) {
          const int r = lane + 64 * t;
          if (r >= j && r < n) q[t] -= w * (r == j ? v0 : v[r]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CR; ++t) {
      const int r = lane + 64 * t;
      if (r < np) Ud[(size_t)r * np + jj] = q[t];
    }
  }
}

// After wg_qrp: U = Q S (columns in pivot order, S = sign(diag R)) into Ud (np x np row-major,
// zero padded), d_j = |R_jj| into dd (1 on padding), then X <- T' = D^{-1} S R P^T in original
// column order, still column-major (zero padded): T'[a][col] = s_a R(a, col) / d_a when
// rank[col] >= a.
// Panel width of the blocked factorisations and the largest padded size they serve.
constexpr int QB = 16;
constexpr int QR_BLOCK_MAX_NP = 2 * NT;


__device__ __noinline__ void q_form_blocked(int n, int np, DQMC_LDS double* stage_lds, double* qrv,
                                            const DQMC_LDS int* ordv, const DQMC_LDS double* vd,
                                            const DQMC_LDS double* bt, const double* X, double* W,
                                            double* Ud);

template <typename WT>
__device__ __forceinline__ void udt_finish(Ctx<WT>& c, double* X, double* Ud, double* dd, int* flags,
                                           double* wfree) {
  const int n = c.n, np = c.np, tid = threadIdx.x;
  if (wfree && c.qrv && c.stage && np <= QR_BLOCK_MAX_NP)
    q_form_blocked(n, np, (DQMC_LDS double*)c.stage, c.qrv, (const DQMC_LDS int*)c.ordv,
                   (const DQMC_LDS double*)c.vd, (const DQMC_LDS double*)c.bt, X, wfree, Ud);
  else if (np <= 128) q_columns<2>(n, np, X, c.vd, c.bt, c.ordv, Ud);
  else if (np <= 256) q_columns<4>(n, np, X, c.vd, c.bt, c.ordv, Ud);
  else if (np <= 512) q_columns<8>(n, np, X, c.vd, c.bt, c.ordv, Ud);
  else if (np <= 1024) q_columns<16>(n, np, X, c.vd, c.bt, c.ordv, Ud);
  else q_columns<32>(n, np, X, c.vd, c.bt, c.ordv, Ud);
  __syncthreads();
  // signs and scales
  for (int jj = tid; jj < np; jj += NT) {
    double dj = 1.0, sj = 1.0;
    if (jj < n) {
      const double rjj = X[(size_t)c.ordv[jj] * np + jj];
      dj = fabs(rjj);
      sj = (rjj < 0.0) ? -1.0 : 1.0;
      if (!(dj > 0.0)) atomicOr(flags, FLAG_SINGULAR);
    }
    c.dtmp[jj] = sj;
    dd[jj] = dj;
  }
  __syncthreads();
  for (int e = tid; e < np * np; e += NT) {
    const int r = e / np, col = e - r * np;
    if (col < n) Ud[e] *= c.dtmp[col];
  }
  for (int e = tid; e < np * np; e += NT) {
    const int col = e / np, aa = e - col * np;    // column-major walk
    double v = 0.0;
    if (aa < n && col < n && c.rank[col] >= aa) v = c.dtmp[aa] * X[e] / dd[aa];
    X[e] = v;
  }
  __syncthreads();
}

// Blocked Householder QR of the N > 64 kernels (matrices in the workspace).  The columns are
// sorted once by decreasing norm instead of being pivoted at every step (QR with pre-pivoting,
// Bai, Lee, Li and Xu, Linear Algebra Appl. 435 (2011) 659: as accurate as column pivoting for
// the graded products of the stabilisation, and it leaves the factorisation free to be blocked).
// Panels of QB columns are factorised with the panel in registers, one workgroup reduction of
// QB values per column (z_q = sum_r a_rj a_rq over the rows still active: the column's norm, the
// projections of the later columns, and the V^T v products of the compact-WY factor).  Each
// panel's reflectors satisfy H_1 ... H_QB = I - V T V^T (Schreiber and Van Loan) with T upper
// triangular, T_jj = beta_j, T(0:j, j) = -beta_j T(0:j, 0:j) V(:, 0:j)^T v_j.  The trailing
// columns get C <- (I - V T^T V^T) C and the explicit Q = H_1 ... H_n is accumulated from the
// last panel back, both as MFMA products.  Outputs as wg_qrp + udt_finish: U = Q S into Ud
// (row-major, zero padded), d = |diag R| into dd (1 on padding), and X <- T' = D^{-1} S R P^T
// column-major in original column order (P the pre-pivot permutation).  A is a scratch matrix.

// Not inlined: it has its own register budget inside the large generic sweep kernel, and one
// instance per RPT serves both working precisions.  LDS arguments carry their address space.
template <int RPT>
__device__ __noinline__ void udt_blocked(int n, int np, DQMC_LDS double* stage_lds, double* qrv,
                                         DQMC_LDS double* nrm, DQMC_LDS int* ordv, DQMC_LDS int* rank,
                                         DQMC_LDS double* vdv, DQMC_LDS double* btv,
                                         DQMC_LDS double* dtmp, double* X, double* A, double* Ud,
                                         double* dd, int* flags) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* V = qrv;                         // reflectors, np x np column-major, zero above the diagonal
  double* Tg = qrv + (size_t)np * np;      // T of panel p at Tg[p QB^2], row-major
  DQMC_LDS double* red = stage_lds;        // [NW][QB] partial sums
  DQMC_LDS double* rowv = red + NW * QB;   // [QB] row r0 of the panel
  // 1. pre-pivot: rank of each column by (norm descending, index ascending), a strict order
  for (int col = wave; col < n; col += NW) {
    double s = 0;
    for (int r = lane; r < n; r += 64) { const double x = X[(size_t)col * np + r]; s += x * x; }
    s = wave_sum_dpp(s);
    if (lane == 0) nrm[col] = (s == s) ? s : -1.0;
  }
  __syncthreads();
  for (int col = tid; col < n; col += NT) {
    const double key = nrm[col];
    int rk = 0;
    for (int c2 = 0; c2 < n; ++c2) {
      const double k2 = nrm[c2];
      rk += (k2 > key || (k2 == key && c2 < col)) ? 1 : 0;
    }
    ordv[rk] = col;
    rank[col] = rk;
  }
  __syncthreads();
  // 2. A = X P (columns in pre-pivot order), V = 0
  for (int e = tid; e < np * np; e += NT) {
    const int j = e / np, r = e - j * np;
    double v = 0.0;
    if (j < n) {
      int src = ordv[j];
      src = (src >= 0 && src < n) ? src : j;
      v = X[(size_t)src * np + r];
    }
    A[e] = v;
    V[e] = 0.0;
  }
  __syncthreads();
  // 3. panels
  for (int k0 = 0, pnl = 0; k0 < n; k0 += QB, ++pnl) {
    const int nbk = min(QB, n - k0);
    // row tid of the panel's T factor (threads tid < QB): T(i, j) depends on row i only
    double trow[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) trow[q] = 0.0;
    double p[RPT][QB];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int r = k0 + tid + NT * m;
#pragma unroll
      for (int q = 0; q < QB; ++q) p[m][q] = (r < np) ? A[(size_t)(k0 + q) * np + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      if (j < nbk) {
        const int r0 = k0 + j;
        double z[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) z[q] = 0.0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
          const int r = k0 + tid + NT * m;
          if (r >= r0 && r < np) {
#pragma unroll
            for (int q = 0; q < QB; ++q) z[q] += p[m][j] * p[m][q];
          }
        }
        if (tid == j) {
#pragma unroll
          for (int q = 0; q < QB; ++q) rowv[q] = p[0][q];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const double t = wave_sum_dpp(z[q]);
          if (lane == 0) red[wave * QB + q] = t;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) t += red[w * QB + q];
          z[q] = t;
        }
        const double x0 = rowv[j];
        const double nx = sqrt(z[j]);
        const double al = (x0 >= 0.0) ? -nx : nx;
        const double be = (nx > 0.0) ? 1.0 / (al * (al - x0)) : 0.0;
        const double v0 = x0 - al;
#pragma unroll
        for (int q = j + 1; q < QB; ++q) {
          const double w = be * (z[q] - al * rowv[q]);
#pragma unroll
          for (int m = 0; m < RPT; ++m) {
            const int r = k0 + tid + NT * m;
            if (r >= r0 && r < np) p[m][q] -= w * ((r == r0) ? v0 : p[m][j]);
          }
        }
        // T(i, j) = -be sum_{k = i}^{j-1} T(i, k) y_k (i < j), T(j, j) = be, y_k = V(:, k)^T v_j
        if (tid < j) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < j; ++k)
            if (k >= tid) acc += trow[k] * (z[k] - al * rowv[k]);
          trow[j] = -be * acc;
        } else if (tid == j) {
          trow[j] = be;
        }
        if (tid == 0) {
          vdv[r0] = al;
          btv[j] = v0;
        }
        if (tid == j) p[0][j] = al;
        __syncthreads();
      }
    }
    // the panel back into A (R above, reflectors below), clean reflectors into V, T out
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int r = k0 + tid + NT * m;
      if (r < np) {
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          A[(size_t)(k0 + q) * np + r] = p[m][q];
          double v = 0.0;
          if (q < nbk) v = (r > k0 + q) ? p[m][q] : ((r == k0 + q) ? btv[q] : 0.0);
          V[(size_t)(k0 + q) * np + r] = v;
        }
      }
    }
    if (tid < QB) {
#pragma unroll
      for (int q = 0; q < QB; ++q) Tg[(size_t)pnl * QB * QB + tid * QB + q] = trow[q];
    }
    __syncthreads();
    // trailing columns: C <- C - V (T^T (V^T C)), W = V^T C staged in Ud (free until step 4)
    if (n - k0 - QB > 0) {
      const int ncr = ((n - k0 - QB) + 15) & ~15;
      double* W = Ud;
      const double* Vp = V + (size_t)k0 * np + k0;
      const double* C = A + (size_t)(k0 + QB) * np + k0;
      wave_gemm<double>(1, QB, ncr, np - k0, Vp, Vp, np, 1, C, C, 1, np,
                       [&](int, int i, int j, double v) { W[(size_t)i * np + j] = v; });
      __syncthreads();
      const double* T = Tg + (size_t)pnl * QB * QB;
      for (int j = tid; j < ncr; j += NT) {
        double w[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) w[q] = W[(size_t)q * np + j];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          double s = 0.0;
#pragma unroll
          for (int b = 0; b <= q; ++b) s += T[b * QB + q] * w[b];
          W[(size_t)q * np + j] = s;
        }
      }
      __syncthreads();
      wave_gemm<double>(1, np - k0, ncr, QB, Vp, Vp, 1, np, W, W, np, 1,
                       [&](int, int i, int j, double v) { A[(size_t)(k0 + QB + j) * np + k0 + i] -= v; });
      __syncthreads();
    }
  }
  // 4. Q = H_1 ... H_n from the last panel back: Q <- Q - V (T (V^T Q)) on rows >= k0; columns
  //    < k0 of the partial product are zero on those rows and are skipped.  W staged in X.
  for (int e = tid; e < np * np; e += NT) {
    const int r = e / np, col = e - r * np;
    Ud[e] = (r == col && r < n) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int pnl = (n + QB - 1) / QB - 1; pnl >= 0; --pnl) {
    const int k0 = pnl * QB, w = np - k0;
    double* W = X;
    const double* Vp = V + (size_t)k0 * np + k0;
    double* Qb = Ud + (size_t)k0 * np + k0;
    wave_gemm<double>(1, QB, w, w, Vp, Vp, np, 1, Qb, Qb, np, 1,
                     [&](int, int i, int j, double v) { W[(size_t)i * np + j] = v; });
    __syncthreads();
    const double* T = Tg + (size_t)pnl * QB * QB;
    for (int j = tid; j < w; j += NT) {
      double t[QB];
#pragma unroll
      for (int q = 0; q < QB; ++q) t[q] = W[(size_t)q * np + j];
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        double s = 0.0;
#pragma unroll
        for (int b = q; b < QB; ++b) s += T[q * QB + b] * t[b];
        W[(size_t)q * np + j] = s;
      }
    }
    __syncthreads();
    wave_gemm<double>(1, w, w, QB, Vp, Vp, 1, np, W, W, np, 1,
                     [&](int, int i, int j, double v) { Qb[(size_t)i * np + j] -= v; });
    __syncthreads();
  }
  // 5. signs and scales, U = Q S, X <- T'
  for (int jj = tid; jj < np; jj += NT) {
    double dj = 1.0, sj = 1.0;
    if (jj < n) {
      const double rjj = vdv[jj];
      dj = fabs(rjj);
      sj = (rjj < 0.0) ? -1.0 : 1.0;
      if (!(dj > 0.0)) atomicOr(flags, FLAG_SINGULAR);
    }
    dtmp[jj] = sj;
    dd[jj] = dj;
  }
  __syncthreads();
  for (int e = tid; e < np * np; e += NT) {
    const int col = e - (e / np) * np;
    if (col < n) Ud[e] *= dtmp[col];
  }
  for (int e = tid; e < np * np; e += NT) {
    const int col = e / np, a = e - col * np;
    double v = 0.0;
    if (col < n && a < n) {
      int j = rank[col];
      j = (j >= 0 && j < n) ? j : col;
      if (a <= j) v = dtmp[a] * A[(size_t)j * np + a] / dd[a];
    }
    X[e] = v;
  }
  __syncthreads();
}

// Explicit Q = H_0 H_1 ... H_{n-1} of the column-pivoted QR (wg_qrp: reflector j in column
// ordv[j] of X below row j, its diagonal element in vd[j], beta_j in bt[j]) by compact-WY panels
// of QB reflectors: V gathered clean into qrv, each panel's T from Y = V_p^T V_p (one small MFMA
// product), then the backward accumulation Q <- (I - V_p T_p V_p^T) Q as in udt_blocked.  The
// same Q as the column-by-column q_columns up to rounding.  W: a free np x np matrix.
__device__ __noinline__ void q_form_blocked(int n, int np, DQMC_LDS double* stage_lds, double* qrv,
                                            const DQMC_LDS int* ordv, const DQMC_LDS double* vd,
                                            const DQMC_LDS double* bt, const double* X, double* W,
                                            double* Ud) {
  const int tid = threadIdx.x;
  double* V = qrv;
  double* Tg = qrv + (size_t)np * np;
  for (int e = tid; e < np * np; e += NT) {
    const int j = e / np, r = e - j * np;
    double v = 0.0;
    if (j < n) {
      if (r == j) {
        v = vd[j];
      } else if (r > j && r < n) {
        int col = ordv[j];
        col = (col >= 0 && col < n) ? col : j;
        v = X[(size_t)col * np + r];
      }
    }
    V[e] = v;
  }
  __syncthreads();
  const int npnl = (n + QB - 1) / QB;
  DQMC_LDS double* Yl = stage_lds;
  DQMC_LDS double* Tl = stage_lds + QB * QB;
  for (int pnl = 0; pnl < npnl; ++pnl) {
    const int k0 = pnl * QB, nbk = min(QB, n - k0);
    const double* Vp = V + (size_t)k0 * np + k0;
    double* Tp = Tg + (size_t)pnl * QB * QB;
    wave_gemm<double>(1, QB, QB, np - k0, Vp, Vp, np, 1, Vp, Vp, 1, np,
                       [&](int, int i, int j, double v) { Tp[i * QB + j] = v; });
    __syncthreads();
    for (int e = tid; e < QB * QB; e += NT) Yl[e] = Tp[e];
    __syncthreads();
    // row i of T on thread i < QB: T(i, j) = -be_j sum_{k = i}^{j-1} T(i, k) Y(k, j) depends on
    // row i alone
    if (tid < QB) {
      double trow[QB];
#pragma unroll
      for (int j = 0; j < QB; ++j) {
        trow[j] = 0.0;
        if (j < nbk) {
          const double be = bt[k0 + j];
          if (tid == j) {
            trow[j] = be;
          } else if (tid < j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k)
              if (k >= tid) acc += trow[k] * Yl[k * QB + j];
            trow[j] = -be * acc;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < QB; ++j) Tl[tid * QB + j] = trow[j];
    }
    __syncthreads();
    for (int e = tid; e < QB * QB; e += NT) Tp[e] = Tl[e];
    __syncthreads();
  }
  for (int e = tid; e < np * np; e += NT) {
    const int r = e / np, col = e - r * np;
    Ud[e] = (r == col && r < n) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int pnl = npnl - 1; pnl >= 0; --pnl) {
    const int k0 = pnl * QB, w = np - k0;
    const double* Vp = V + (size_t)k0 * np + k0;
    double* Qb = Ud + (size_t)k0 * np + k0;
    wave_gemm<double>(1, QB, w, w, Vp, Vp, np, 1, Qb, Qb, np, 1,
                       [&](int, int i, int j, double v) { W[(size_t)i * np + j] = v; });
    __syncthreads();
    const double* T = Tg + (size_t)pnl * QB * QB;
    for (int j = tid; j < w; j += NT) {
      double t[QB];
#pragma unroll
      for (int q = 0; q < QB; ++q) t[q] = W[(size_t)q * np + j];
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        double s2 = 0.0;
#pragma unroll
        for (int b = q; b < QB; ++b) s2 += T[q * QB + b] * t[b];
        W[(size_t)q * np + j] = s2;
      }
    }
    __syncthreads();
    wave_gemm<double>(1, w, w, QB, Vp, Vp, 1, np, W, W, np, 1,
                       [&](int, int i, int j, double v) { Qb[(size_t)i * np + j] -= v; });
    __syncthreads();
  }
}

// Multiply a chunk of slice propagators onto (Us, ds, Ts) and re-factorise:
//   left  (right == false): product B_{hi} ... B_{lo+1} U D, B_l = V_l expK;
//   right (right == true):  product B_{lo+1}^T ... B_{hi}^T U D, B_l^T = expK^T V_l;
// then UDT of the result: Ud Diag(dd) (T' Ts) -> (Ud, dd, Td).  Ts may be the identity.
// Work matrices w1/w2 are used; the result ends up in the destination buffers.
template <typename WT>
__device__ __forceinline__ void udt_push(Ctx<WT>& c, int spin, bool right, int lo, int hi, const double* Us,
                         const double* ds, const double* Ts, double* Ud, double* dd, double* Td) {
  PhaseClock pc;
  pc.start();
  const KArgs& a = *c.a;
  const int np = c.np, n = c.n;
  double* cur = c.w1;
  double* nxt = c.w2;
  if (!right) {
    form_ud(np, Us, ds, nullptr, cur);
    __syncthreads();
    for (int l = lo + 1; l <= hi; ++l) {
      const int8_t* fl = c.f + (size_t)(l - 1) * np;
      const bool last = (l == hi);   // the last product goes out column-major for the QR
      ctx_gemm<double>(c, 1, np, np, np, a.expK, a.expK, np, 1, cur, cur, np, 1,
                      [&](int, int i, int j, double v) {
                        double s = (i < n) ? vfac(a, spin, fl[i]) : 1.0;
                        nxt[last ? (size_t)j * np + i : (size_t)i * np + j] = s * v;
                      });
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
  } else {
    // X0 = V_hi U D
    {
      const int8_t* fl = c.f + (size_t)(hi - 1) * np;
      for (int e = threadIdx.x; e < np * np; e += NT) {
        int i = e / np, j = e - i * np;
        double s = (i < n) ? vfac(a, spin, fl[i]) : 1.0;
        cur[e] = s * Us[e] * ds[j];
      }
    }
    __syncthreads();
    for (int l = hi; l >= lo + 1; --l) {
      const int8_t* fn = (l - 1 >= lo + 1) ? c.f + (size_t)(l - 2) * np : nullptr;
      // expK^T as the A operand: A(i,k) = expK[k*np + i]
      const bool last = (l == lo + 1);
      ctx_gemm<double>(c, 1, np, np, np, a.expK, a.expK, 1, np, cur, cur, np, 1,
                      [&](int, int i, int j, double v) {
                        double s = (fn && i < n) ? vfac(a, spin, fn[i]) : 1.0;
                        nxt[last ? (size_t)j * np + i : (size_t)i * np + j] = s * v;
                      });
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
  }
  pc.stop(c.st, PH_CHUNK);
  if (a.qr_blocked && c.qrv && c.stage && np <= QR_BLOCK_MAX_NP) {
    DQMC_LDS double* stg = (DQMC_LDS double*)c.stage;
    DQMC_LDS double* nrm = (DQMC_LDS double*)c.nrm;
    DQMC_LDS int* ordv = (DQMC_LDS int*)c.ordv;
    DQMC_LDS int* rnk = (DQMC_LDS int*)c.rank;
    DQMC_LDS double* vdv = (DQMC_LDS double*)c.vd;
    DQMC_LDS double* btv = (DQMC_LDS double*)c.bt;
    DQMC_LDS double* dtm = (DQMC_LDS double*)c.dtmp;
    if (np <= NT) udt_blocked<1>(n, np, stg, c.qrv, nrm, ordv, rnk, vdv, btv, dtm, cur, nxt, Ud, dd, &c.st->flags);
    else udt_blocked<2>(n, np, stg, c.qrv, nrm, ordv, rnk, vdv, btv, dtm, cur, nxt, Ud, dd, &c.st->flags);
    pc.stop(c.st, PH_QR);
  } else {
    if (c.stage && np <= QR_BLOCK_MAX_NP) {
      DQMC_LDS double* nrm = (DQMC_LDS double*)c.nrm;
      DQMC_LDS int* rnk = (DQMC_LDS int*)c.rank;
      DQMC_LDS int* ordv = (DQMC_LDS int*)c.ordv;
      DQMC_LDS double* vb = (DQMC_LDS double*)c.sc;
      DQMC_LDS double* vdv = (DQMC_LDS double*)c.vd;
      DQMC_LDS double* btv = (DQMC_LDS double*)c.bt;
      DQMC_LDS double* rv = (DQMC_LDS double*)c.red.v;
      DQMC_LDS int* ri = (DQMC_LDS int*)c.red.i;
      if (np <= 128) qrp_columns<2>(n, np, cur, nrm, rnk, ordv, vb, vdv, btv, rv, ri);
      else if (np <= 256) qrp_columns<4>(n, np, cur, nrm, rnk, ordv, vb, vdv, btv, rv, ri);
      else qrp_columns<8>(n, np, cur, nrm, rnk, ordv, vb, vdv, btv, rv, ri);
    } else {
      wg_qrp(c, cur);
    }
    pc.stop(c.st, PH_QR);
    udt_finish(c, cur, Ud, dd, &c.st->flags, nxt);
    pc.stop(c.st, PH_QFORM);
  }
  // Td = T' Ts  (cur now holds T', column-major)
  ctx_gemm<double>(c, 1, np, np, np, cur, cur, 1, np, Ts, Ts, np, 1,
                  [&](int, int i, int j, double v) { Td[i * np + j] = v; });
  __syncthreads();
  pc.stop(c.st, PH_TMUL);
}

// ------------------------------------------------------------------------------ fresh G
// Gauss-Jordan elimination with partial (implicit) row pivoting on M (n x n, leading dim np),
// applied to the right-hand side Z (np columns).  On return w_dst = M^{-1} Z with its rows
// scaled by rs[] (rs may be null), and the log|det M| is returned to all threads.  The pivot
// row is staged in LDS; one wavefront per eliminated row, its lanes along the row.
template <typename WT>
__device__ __forceinline__ double wg_gauss_jordan(Ctx<WT>& c, double* M, double* Z, double* dst, const double* rs) {
  const int n = c.n, np = c.np, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* prow = c.sr;   // [2 np]: M[p][j+1 .. n-1] then Z[p][0 .. np-1]
  for (int k = tid; k < np; k += NT) c.rank[k] = -1;   // rank[row] = step at which row pivoted
  __syncthreads();
  double logabs = 0.0;
  for (int j = 0; j < n; ++j) {
    double key = -1.0;
    int idx = -1;
    for (int r = tid; r < n; r += NT) {
      if (c.rank[r] < 0) {
        const double v = fabs(M[(size_t)r * np + j]);
        if (idx < 0 || v > key) { key = v; idx = r; }
      }
    }
    const int p = wg_argmax(key, idx, c.red);
    const double piv = M[(size_t)p * np + j];
    logabs += log(fabs(piv));
    const int wM = n - j - 1;   // columns j+1 .. n-1 of M
    for (int e = tid; e < wM + np; e += NT)
      prow[e] = (e < wM) ? M[(size_t)p * np + j + 1 + e] : Z[(size_t)p * np + (e - wM)];
    if (tid == 0) { c.rank[p] = j; c.ordv[j] = p; c.dtmp[j] = piv; }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int r = wave; r < n; r += NW) {
      if (r == p) continue;
      double* mr = M + (size_t)r * np;
      const double fct = mr[j] * inv;
      if (fct == 0.0) continue;
      for (int e = lane; e < wM; e += 64) mr[j + 1 + e] -= fct * prow[e];
      double* zr = Z + (size_t)r * np;
      for (int e = lane; e < np; e += 64) zr[e] -= fct * prow[wM + e];
    }
    __syncthreads();
  }
  // x_j = Z[ordv[j]] / pivot_j, rows scaled by rs
  for (int e = tid; e < np * np; e += NT) {
    const int j = e / np, col = e - j * np;
    double v = 0.0;
    if (j < n) {
      v = Z[(size_t)c.ordv[j] * np + col] / c.dtmp[j];
      if (rs) v *= rs[j];
    }
    dst[e] = v;
  }
  __syncthreads();
  return logabs;
}

// Blocked Gauss-Jordan solve of the N > 64 kernels: dst = Diag(rs) M^{-1} Z with the same
// partial (implicit) row pivoting as wg_gauss_jordan, QB columns at a time.  For a panel K of
// columns with pivot rows P (chosen in registers, one row per thread, by eliminating the panel on
// the rows not yet pivoted) the Gauss-Jordan steps of the panel act on every other column as
//   rows r not in P:  x_r <- x_r - M[r, K] A_P^{-1} x_P,     rows P:  x_P <- A_P^{-1} x_P,
// A_P = M[P, K] (rows in pivot order; its elimination without further pivoting is the panel's
// partially pivoted one), so the later columns of M and all of Z take one rank-QB MFMA update
// per panel.  Afterwards row ordv[j] of Z holds solution row j.  Returns log|det M| (the sum of
// the logs of the pivots) to every thread.  scr: QB np + QB 2np doubles of workspace.
template <int RPT>
__device__ __noinline__ double gj_blocked(int n, int np, DQMC_LDS double* stage_lds, double* scr,
                                          DQMC_LDS int* ordv, DQMC_LDS int* rank,
                                          const DQMC_LDS double* rs, double* M, double* Z,
                                          double* dst) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  DQMC_LDS double* red = stage_lds;                     // [NW] argmax keys
  DQMC_LDS int* redi = (DQMC_LDS int*)(red + NW);       // [NW] argmax rows
  DQMC_LDS double* prow = red + 2 * NW;                 // [QB] pivot row, panel part
  DQMC_LDS double* Ap = prow + QB;                      // [QB][QB] A_P, then eliminated
  DQMC_LDS double* Ai = Ap + QB * QB;                   // [QB][QB] A_P^{-1}
  const int ldw = 2 * np;
  double* Qp = scr;                                     // np x QB: M[r, K], zero on rows P
  double* W = scr + (size_t)np * QB;                    // QB x ldw: A_P^{-1} [M[P, later] | Z[P, :]]
  for (int k = tid; k < np; k += NT) rank[k] = -1;
  __syncthreads();
  double logabs = 0.0;
  for (int k0 = 0; k0 < n; k0 += QB) {
    const int nbk = min(QB, n - k0);
    double p[RPT][QB], q[RPT][QB];
    int rk[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int r = tid + NT * m;
      rk[m] = (r < n) ? rank[r] : 0;
#pragma unroll
      for (int c = 0; c < QB; ++c) {
        const double v = (r < n && c < nbk) ? M[(size_t)r * np + k0 + c] : 0.0;
        p[m][c] = v;
        q[m][c] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      if (j < nbk) {
        // pivot: largest |value| in column j among rows not yet pivoted (NaN counts as -0.5,
        // so a row is always found); ties go to the lower row
        double key = -1.0;
        int idx = -1;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
          const int r = tid + NT * m;
          if (r < n && rk[m] < 0) {
            double v = fabs(p[m][j]);
            v = (v == v) ? v : -0.5;
            if (idx < 0 || v > key) { key = v; idx = r; }
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double k2 = __shfl_xor(key, o);
          const int i2 = __shfl_xor(idx, o);
          if (i2 >= 0 && (idx < 0 || k2 > key || (k2 == key && i2 < idx))) { key = k2; idx = i2; }
        }
        if (lane == 0) { red[wave] = key; redi[wave] = idx; }
        __syncthreads();
        double bk = red[0];
        int pr = redi[0];
        for (int w = 1; w < NW; ++w) {
          const double k2 = red[w];
          const int i2 = redi[w];
          if (i2 >= 0 && (pr < 0 || k2 > bk || (k2 == bk && i2 < pr))) { bk = k2; pr = i2; }
        }
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
          if (pr == tid + NT * m) {
#pragma unroll
            for (int c = 0; c < QB; ++c) {
              prow[c] = p[m][c];
              Ap[j * QB + c] = q[m][c];
            }
            rank[pr] = k0 + j;
            ordv[k0 + j] = pr;
            rk[m] = k0 + j;
          }
        }
        __syncthreads();
        const double piv = prow[j];
        logabs += log(fabs(piv));
        const double ipiv = 1.0 / piv;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
          const int r = tid + NT * m;
          if (r < n && rk[m] < 0) {
            const double f = p[m][j] * ipiv;
#pragma unroll
            for (int c = j + 1; c < QB; ++c) p[m][c] -= f * prow[c];
          }
        }
        __syncthreads();
      }
    }
    // Qp = M[:, K] with the rows of P zeroed
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int r = tid + NT * m;
      if (r < np) {
        const bool inP = (r < n) && rk[m] >= k0;
#pragma unroll
        for (int c = 0; c < QB; ++c) Qp[(size_t)r * QB + c] = inP ? 0.0 : q[m][c];
      }
    }
    // A_P^{-1} by Gauss-Jordan without pivoting (identity on the padding of a short panel)
    {
      const int r = tid >> 4, c = tid & 15;   // NT = 256 = QB * QB entries
      if (r >= nbk || c >= nbk) Ap[r * QB + c] = (r == c) ? 1.0 : 0.0;
      Ai[r * QB + c] = (r == c) ? 1.0 : 0.0;
      __syncthreads();
      for (int s2 = 0; s2 < QB; ++s2) {
        const double d = Ap[s2 * QB + s2];
        const double fr = Ap[r * QB + s2];
        const double as = Ap[s2 * QB + c], is = Ai[s2 * QB + c];
        const double ar = Ap[r * QB + c], ir = Ai[r * QB + c];
        __syncthreads();
        if (r == s2) {
          Ap[r * QB + c] = as / d;
          Ai[r * QB + c] = is / d;
        } else {
          Ap[r * QB + c] = ar - fr * as / d;
          Ai[r * QB + c] = ir - fr * is / d;
        }
        __syncthreads();
      }
    }
    // W = A_P^{-1} [M[P, k0+QB .. n) | Z[P, :]]
    const int nm = n - k0 - QB;
    const int nmr = nm > 0 ? ((nm + 15) & ~15) : 0;
    for (int col = tid; col < nmr + np; col += NT) {
      double x[QB];
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        double v = 0.0;
        if (b < nbk) {
          const int row = ordv[k0 + b];
          v = (col < nmr) ? M[(size_t)row * np + k0 + QB + col] : Z[(size_t)row * np + (col - nmr)];
        }
        x[b] = v;
      }
#pragma unroll
      for (int a = 0; a < QB; ++a) {
        double s2 = 0.0;
#pragma unroll
        for (int b = 0; b < QB; ++b) s2 += Ai[a * QB + b] * x[b];
        W[(size_t)a * ldw + col] = s2;
      }
    }
    __syncthreads();
    // rows not in P: x -= M[r, K] W;  rows in P: x = W (their Qp rows are zero)
    if (nmr > 0) {
      wave_gemm<double>(1, np, nmr, QB, Qp, Qp, QB, 1, W, W, ldw, 1,
                         [&](int, int i, int j, double v) {
                           const int rr = rank[i];
                           double* e = M + (size_t)i * np + k0 + QB + j;
                           if (rr >= k0 && rr < k0 + QB) *e = W[(size_t)(rr - k0) * ldw + j];
                           else *e -= v;
                         });
    }
    wave_gemm<double>(1, np, np, QB, Qp, Qp, QB, 1, W + nmr, W + nmr, ldw, 1,
                       [&](int, int i, int j, double v) {
                         const int rr = rank[i];
                         double* e = Z + (size_t)i * np + j;
                         if (rr >= k0 && rr < k0 + QB) *e = W[(size_t)(rr - k0) * ldw + nmr + j];
                         else *e -= v;
                       });
    __syncthreads();
  }
  // solution row j sits in row ordv[j] of Z
  for (int e = tid; e < np * np; e += NT) {
    const int j = e / np, col = e - j * np;
    double v = 0.0;
    if (j < n) {
      int row = ordv[j];
      row = (row >= 0 && row < n) ? row : j;
      v = Z[(size_t)row * np + col];
      if (rs) v *= rs[j];
    }
    dst[e] = v;
  }
  __syncthreads();
  return logabs;
}

// Fresh equal-time G^spin = [I + A B]^{-1} with A = UL DL TL (left, B(l,0)) and
// B^T = UR DR TR (right, B(L,l)^T), by the two-sided split of the scales at 1:
//   d = db ds, db = max(d,1), ds = min(d,1);
//   I + A B = UL DLb [DLb^{-1} UL^T UR DRb^{-1} + DLs TL TR^T DRs] DRb UR^T = UL DLb M DRb UR^T
//   G = UR DRb^{-1} M^{-1} DLb^{-1} UL^T,  log|det(I + A B)| = sum log DLb + sum log DRb + log|det M|.
// The result replaces c.G[spin] (and G64 when g64 != null); returns the drift
// max|G_old - G_new| and writes log|det| into *logdet.
template <typename WT>
__device__ __forceinline__ double fresh_green(Ctx<WT>& c, int spin, const double* UL, const double* dL,
                              const double* TL, const double* UR, const double* dR,
                              const double* TR, double* g64, double* logdet, bool drift) {
  const int np = c.np, n = c.n, tid = threadIdx.x;
  PhaseClock pc;
  pc.start();
  double* M = c.w1;
  double* Z = c.w2;
  // sr <- 1/DLb, sc <- 1/DRb for this call (slice scales are not live here)
  double* iLb = c.sr;
  double* iRb = c.sc;
  for (int i = tid; i < np; i += NT) {
    iLb[i] = 1.0 / fmax(dL[i], 1.0);
    iRb[i] = 1.0 / fmax(dR[i], 1.0);
  }
  __syncthreads();
  // M = DLb^{-1} (UL^T UR) DRb^{-1};  Z = DLb^{-1} UL^T
  ctx_gemm<double>(c, 1, np, np, np, UL, UL, 1, np, UR, UR, np, 1,
                  [&](int, int i, int j, double v) { M[i * np + j] = v * iLb[i] * iRb[j]; });
  for (int e = tid; e < np * np; e += NT) {
    int i = e / np, j = e - i * np;
    Z[e] = UL[j * np + i] * iLb[i];
  }
  __syncthreads();
  // M += DLs (TL TR^T) DRs
  ctx_gemm<double>(c, 1, np, np, np, TL, TL, np, 1, TR, TR, 1, np, [&](int, int i, int j, double v) {
    M[i * np + j] += fmin(dL[i], 1.0) * v * fmin(dR[j], 1.0);
  });
  __syncthreads();
  pc.stop(c.st, PH_FGEMM);
  // Z <- DRb^{-1} M^{-1} DLb^{-1} UL^T  (written into M's buffer)
  double logm;
  if (c.qrv && c.stage && np <= QR_BLOCK_MAX_NP) {
    DQMC_LDS double* stg = (DQMC_LDS double*)c.stage;
    DQMC_LDS int* ordv = (DQMC_LDS int*)c.ordv;
    DQMC_LDS int* rnk = (DQMC_LDS int*)c.rank;
    const DQMC_LDS double* rsv = (const DQMC_LDS double*)iRb;
    logm = (np <= NT) ? gj_blocked<1>(n, np, stg, c.qrv, ordv, rnk, rsv, M, Z, M)
                      : gj_blocked<2>(n, np, stg, c.qrv, ordv, rnk, rsv, M, Z, M);
  } else {
    logm = wg_gauss_jordan(c, M, Z, M, iRb);
  }
  pc.stop(c.st, PH_GJ);
  // G = UR (DRb^{-1} M^{-1} DLb^{-1} UL^T)
  WT* G = c.G[spin];
  double dmax = 0.0;
  bool bad = false;
  ctx_gemm<double>(c, 1, np, np, np, UR, UR, np, 1, M, M, np, 1, [&](int, int i, int j, double v) {
    const int e = i * np + j;
    if (drift) dmax = fmax(dmax, fabs((double)G[e] - v));
    if (!(fabs(v) < 1e300)) bad = true;
    G[e] = (WT)v;
    if (g64) g64[e] = v;
  });
  if (bad) atomicOr(&c.st->flags, FLAG_NONFINITE);
  pc.stop(c.st, PH_GOUT);
  double ld = logm;
  {
    double part = 0.0;
    for (int i = tid; i < n; i += NT) part += log(fmax(dL[i], 1.0)) + log(fmax(dR[i], 1.0));
    part = wave_sum(part);
    double* buf = c.red.v + c.red.parity * NW;
    c.red.parity ^= 1;
    if ((tid & 63) == 0) buf[tid >> 6] = part;
    __syncthreads();
    for (int w = 0; w < NW; ++w) ld += buf[w];
  }
  *logdet = ld;
  double dr = drift ? wg_max(dmax, c.red) : 0.0;
  return dr;
}

// ------------------------------------------------------------------------------ wrap
// G^sigma(l) = B_l G^sigma(l-1) B_l^{-1} = V_l expK G expKinv V_l^{-1} for both spins:
// two MFMA products per spin in the working precision, the diagonal factors in the epilogue.
template <typename WT>
__device__ __forceinline__ void wrap_both(Ctx<WT>& c, int l) {
  const KArgs& a = *c.a;
  const int np = c.np;
  slice_scales(c, l - 1);
  WT* t0 = (WT*)c.w1;
  WT* t1 = (WT*)c.w2;
  const WT* K1 = kexp<WT>(a);
  const WT* K2 = kexpinv<WT>(a);
  ctx_gemm<WT>(c, 2, np, np, np, K1, K1, np, 1, c.G[0], c.G[1], np, 1,
              [&](int b, int i, int j, WT v) { (b ? t1 : t0)[i * np + j] = v; });
  __syncthreads();
  ctx_gemm<WT>(c, 2, np, np, np, t0, t1, np, 1, K2, K2, np, 1, [&](int b, int i, int j, WT v) {
    c.G[b][i * np + j] = (WT)(c.sr[b * np + i] * (double)v * c.sc[b * np + j]);
  });
  __syncthreads();
}

// G(l-1) = B_l^{-1} G(l) B_l = e^{+dtau T} V_l^{-1} G(l) V_l e^{-dtau T} for both spins (down
// sweeps): the diagonal factors in place, then two MFMA products.
template <typename WT>
__device__ __forceinline__ void unwrap_both(Ctx<WT>& c, int l) {
  const KArgs& a = *c.a;
  const int np = c.np;
  slice_scales(c, l - 1);
  __syncthreads();   // the scales are read by every thread below
  for (int e = threadIdx.x; e < 2 * np * np; e += NT) {
    const int b = e / (np * np), r = e - b * (np * np), i = r / np, j = r - i * np;
    c.G[b][r] = (WT)(c.sc[b * np + i] * (double)c.G[b][r] * c.sr[b * np + j]);
  }
  __syncthreads();
  WT* t0 = (WT*)c.w1;
  WT* t1 = (WT*)c.w2;
  const WT* K1 = kexp<WT>(a);
  const WT* K2 = kexpinv<WT>(a);
  ctx_gemm<WT>(c, 2, np, np, np, K2, K2, np, 1, c.G[0], c.G[1], np, 1,
               [&](int b, int i, int j, WT v) { (b ? t1 : t0)[i * np + j] = v; });
  __syncthreads();
  ctx_gemm<WT>(c, 2, np, np, np, t0, t1, np, 1, K1, K1, np, 1,
               [&](int b, int i, int j, WT v) { c.G[b][i * np + j] = v; });
  __syncthreads();
}

// ------------------------------------------------------------------------------ Metropolis
// Single-flip Metropolis over the sites of slice l with submatrix (delayed) updates.
//
// Flipping s_{i,l} multiplies B^sigma_l from the left by (I + Delta^sigma e_i e_i^T),
// Delta^sigma = e^{-2 sigma nu s_{i,l}} - 1, so with G = G(l) the weight ratio is
// R = prod_sigma (1 + Delta^sigma (1 - G^sigma_ii)) and, on acceptance,
// G' = G (I + Delta (I - G))^{-1} = G - (Delta/R^sigma) G[:,i] (e_i - G[i,:])  (Sherman-Morrison).
// Sites are taken in blocks B of K consecutive sites.  Within a block only G[B,B] is needed to
// decide, so one wavefront runs the block sequentially on a K x K copy (no workgroup barrier),
// recording for the m-th accepted flip at site j_m
//     x_m = -(Delta/R) G_{m-1}[:, j_m],   y_m = e_{j_m} - G_{m-1}[j_m, :]   (block entries),
// so that after the block G = G0 + X Y with the full columns/rows obtained row by row from
//     X[r,m] = -(Delta_m/R_m) (G0[r, j_m] + sum_{m'<m} X[r,m'] Y[m', j_m])
//     Y[m,c] = delta_{c,j_m} - G0[j_m, c] - sum_{m'<m} X[j_m, m'] Y[m', c]
// and the rank-m correction applied as one MFMA product.
// One wavefront decides the kb sites i0 .. i0+kb-1 of slice l in order, with the block of the
// true G of both spins in c.gb: ratio, Philox uniform, Metropolis test, and on acceptance the
// block's own rank-1 update and the block parts of the Sherman-Morrison vectors (x_m rows in xb,
// y_m columns in yb, both spins), the accepted site, its two coefficients and the field flip.
// The number accepted goes to c.cnt[(i0 / K) % 2] (two words used in turn: after a block with no
// accepts no barrier separates the other waves' read of its count from the next block's write);
// log|R| per spin is added to ldrun.  Run by wave 0.
template <typename WT>
__device__ __forceinline__ void decide_block(Ctx<WT>& c, int l, int i0, int kb, uint64_t seed,
                                             int64_t sweep, int8_t* fl, double* ldrun) {
  const KArgs& a = *c.a;
  const int K = c.K, K2 = K * K, lane = threadIdx.x & 63;
  if (lane < kb) {
    c.ublk[lane] = accept_uniform(seed, sweep, l - 1, i0 + lane);
    c.sblk[lane] = fl[i0 + lane];
  }
  wave_sync();
  int m = 0;
  double ldu = 0.0, ldd = 0.0;
  int flg = 0;
  int64_t ties = 0;
  for (int ii = 0; ii < kb; ++ii) {
    const int s = c.sblk[ii];
    const double u = c.ublk[ii];
    const double gu = c.gb[ii * K + ii], gd = c.gb[K2 + ii * K + ii];
    const double du = a.dup[s > 0], dd = a.ddn[s > 0];
    const double ru = 1.0 + du * (1.0 - gu), rd = 1.0 + dd * (1.0 - gd);
    const double R = ru * rd;
    bool ok = true;
    if (!(fabs(R) < 1e300)) { flg |= FLAG_NONFINITE; ok = false; }
    else if (R < 0.0) { flg |= FLAG_NEGATIVE; ok = false; }
    if (ok && fabs(u - R) < 1e-9) ++ties;
    if (ok && u < R) {
      const double cu = du / ru, cd = dd / rd;
      if (lane < kb) {
        const int r = lane;
        c.xb[r * K + m] = -cu * c.gb[r * K + ii];
        c.xb[K2 + r * K + m] = -cd * c.gb[K2 + r * K + ii];
        c.yb[m * K + r] = (r == ii ? 1.0 : 0.0) - c.gb[ii * K + r];
        c.yb[K2 + m * K + r] = (r == ii ? 1.0 : 0.0) - c.gb[K2 + ii * K + r];
      }
      wave_sync();
      // rank-1 update of the block: lane -> column lane % cw, rows lane / cw + k (64 / cw), with
      // cw = 16 or 32 >= kb, so no division per element
      const int cw = (kb <= 16) ? 16 : 32;
      const int cc = lane & (cw - 1), rstep = 64 / cw;
      if (cc < kb) {
        const double yu = c.yb[m * K + cc], yd = c.yb[K2 + m * K + cc];
        for (int r = lane / cw; r < kb; r += rstep) {
          c.gb[r * K + cc] += c.xb[r * K + m] * yu;
          c.gb[K2 + r * K + cc] += c.xb[K2 + r * K + m] * yd;
        }
      }
      if (lane == 0) {
        c.site[m] = ii;
        c.cfu[m] = cu;
        c.cfd[m] = cd;
        fl[i0 + ii] = (int8_t)(-s);
      }
      ldu += log(fabs(ru));
      ldd += log(fabs(rd));
      ++m;
      wave_sync();
    }
  }
  if (lane == 0) {
    c.cnt[(i0 / K) & 1] = m;
    ldrun[0] += ldu;
    ldrun[1] += ldd;
    if (flg) atomicOr(&c.st->flags, flg);
    c.st->near_ties += ties;
  }
}

// Sherman-Morrison vectors of a block's m accepted flips (sites j_t = i0 + site[t], t < m <=
// SM_KMAX, the largest delay rank of the generic kernels), at one row r of X or column r of Y:
//   x_t = -cf_t (g_t + sum_{t2 < t} x_t2 yb[t2][j_t]),       g_t = G(r, j_t)
//   y_t = [r = j_t] - g_t - sum_{t2 < t} xb[j_t][t2] y_t2,   g_t = G(j_t, r)   (0 for r >= n)
// v holds g_t on entry and the vector on exit.  The loops are unrolled to SM_KMAX so that v stays
// in registers (a run-time-indexed array would live in scratch memory) and the caller's loads of
// g are all in flight together; the operations and their order are those of the plain loops.
constexpr int SM_KMAX = 32;
__device__ __forceinline__ void sm_vec_x(int m, const int* site, const double* cf, const double* ybs,
                                         int K, double (&v)[SM_KMAX]) {
#pragma unroll
  for (int t = 0; t < SM_KMAX; ++t) {
    if (t < m) {
      const int jt = site[t];
      double acc = v[t];
#pragma unroll
      for (int t2 = 0; t2 < t; ++t2) acc += v[t2] * ybs[t2 * K + jt];
      v[t] = -cf[t] * acc;
    }
  }
}
__device__ __forceinline__ void sm_vec_y(int m, int r, int i0, int n, const int* site,
                                         const double* xbs, int K, double (&v)[SM_KMAX]) {
#pragma unroll
  for (int t = 0; t < SM_KMAX; ++t) {
    if (t < m) {
      const int jt = site[t];
      double acc = ((r == i0 + jt) ? 1.0 : 0.0) - v[t];
#pragma unroll
      for (int t2 = 0; t2 < t; ++t2) acc -= xbs[jt * K + t2] * v[t2];
      if (r >= n) acc = 0.0;
      v[t] = acc;
    }
  }
}

template <typename WT>
__device__ __forceinline__ void metropolis_slice(Ctx<WT>& c, int l, double* ldrun) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np, K = c.K, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int K2 = K * K;
  int8_t* fl = c.f + (size_t)(l - 1) * np;
  const uint64_t seed = c.st->seed;
  const int64_t sweep = c.st->sweeps_done;
  int64_t acc_total = 0;
  PhaseClock clk;
  clk.start();
  for (int i0 = 0; i0 < n; i0 += K) {
    const int kb = min(K, n - i0);
    if (wave == 0) {
      // ---- phase 1: one wavefront decides the block
      for (int e = lane; e < kb * kb; e += 64) {
        int r = e / kb, cc = e - r * kb;
        c.gb[r * K + cc] = (double)c.G[0][(i0 + r) * np + i0 + cc];
        c.gb[K2 + r * K + cc] = (double)c.G[1][(i0 + r) * np + i0 + cc];
      }
      decide_block(c, l, i0, kb, seed, sweep, fl, ldrun);
    }
    __syncthreads();
    clk.stop(c.st, PH_DECIDE);
    const int m = c.cnt[(i0 / K) & 1];
    acc_total += m;
    if (m == 0) continue;
    const int mp = (m + 3) & ~3;
    // ---- phase 2: full panels X (np x mp, column-major) and Y (mp x np, row-major), both spins
    {
      WT* X0 = c.xy;
      WT* Y0 = c.xy + (size_t)np * K;
      WT* X1 = c.xy + 2 * (size_t)np * K;
      WT* Y1 = c.xy + 3 * (size_t)np * K;
      for (int e = tid; e < 4 * np; e += NT) {
        const int kind = e / (2 * np);          // 0: X rows, 1: Y columns
        const int sp = (e / np) & 1;
        const int r = e - (e / np) * np;        // row (X) or column (Y)
        const WT* G0 = c.G[sp];
        const double* cf = sp ? c.cfd : c.cfu;
        const double* xbs = c.xb + sp * K2;
        const double* ybs = c.yb + sp * K2;
        double v[SM_KMAX];
#pragma unroll
        for (int t = 0; t < SM_KMAX; ++t) {
          v[t] = 0.0;
          if (t < m && r < n)
            v[t] = (double)(kind == 0 ? G0[r * np + i0 + c.site[t]] : G0[(i0 + c.site[t]) * np + r]);
        }
        if (kind == 0) sm_vec_x(m, c.site, cf, ybs, K, v);
        else sm_vec_y(m, r, i0, n, c.site, xbs, K, v);
        WT* P = kind == 0 ? (sp ? X1 : X0) : (sp ? Y1 : Y0);
#pragma unroll
        for (int t = 0; t < SM_KMAX; ++t)
          if (t < mp) P[t * np + r] = (t < m) ? (WT)v[t] : (WT)0;
      }
    }
    __syncthreads();
    clk.stop(c.st, PH_PANEL);
    // ---- phase 3: G += X Y (rank mp) for both spins
    {
      WT* X0 = c.xy;
      WT* Y0 = c.xy + (size_t)np * K;
      WT* X1 = c.xy + 2 * (size_t)np * K;
      WT* Y1 = c.xy + 3 * (size_t)np * K;
      if (c.stage)
        wave_gemm_add<WT>(2, np, np, mp, X0, X1, 1, np, Y0, Y1, np, 1, c.G[0], c.G[1], np);
      else
        ctx_gemm<WT>(c, 2, np, np, mp, X0, X1, 1, np, Y0, Y1, np, 1,
                     [&](int b, int i, int j, WT v) { c.G[b][i * np + j] += v; });
    }
    __syncthreads();
    clk.stop(c.st, PH_FLUSH);
  }
  if (tid == 0) {
    c.st->attempted += n;
    c.st->accepted += acc_total;
  }
}

// Delayed updates in two levels for the matrices in the workspace: blocks of K sites are decided
// as in metropolis_slice, but their accepted flips are appended to accumulated panels XA
// (np x KT, column-major) and YA (KT x np, row-major) instead of entering G at once; the true
// Green's function is G + XA YA.  A block reads its own entries, and the columns and rows of its
// accepted sites, through that correction (small MFMA products), so the decisions and the new
// Sherman-Morrison vectors are those of the one-level scheme; G takes the accumulated rank in one
// product when the panels are full and at the end of the slice.  This replaces one pass over G
// in HBM per block by one per KT / K blocks.
template <typename WT>
__device__ __forceinline__ void metropolis_slice2(Ctx<WT>& c, int l, double* ldrun) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np, K = c.K, KT = a.KT, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int K2 = K * K, K16 = (K + 15) & ~15;
  int8_t* fl = c.f + (size_t)(l - 1) * np;
  const uint64_t seed = c.st->seed;
  const int64_t sweep = c.st->sweeps_done;
  int64_t acc_total = 0;
  const size_t pn = (size_t)np * KT;
  WT* XA[2] = {c.xy, c.xy + pn};
  WT* YA[2] = {c.xy + 2 * pn, c.xy + 3 * pn};
  WT* base = c.xy + 4 * pn;
  WT* Cc[2] = {base, base + (size_t)np * K16};                       // np x K16, column-major
  WT* Rw[2] = {base + 2 * (size_t)np * K16, base + 3 * (size_t)np * K16};   // K16 x np, row-major
  base += 4 * (size_t)np * K16;
  WT* Ys[2] = {base, base + (size_t)KT * K16};                       // KT x K16: YA[u][a_t]
  WT* Xs[2] = {base + 2 * (size_t)KT * K16, base + 3 * (size_t)KT * K16};   // K16 x KT: XA[a_t][u]
  int mA = 0;
  PhaseClock clk;
  clk.start();
  for (int i0 = 0; i0 < n; i0 += K) {
    const int kb = min(K, n - i0);
    // ---- the block of the true G
    if (mA > 0) {
      const int kr = (kb + 15) & ~15;
      wave_gemm<WT>(2, kr, kr, mA, XA[0] + i0, XA[1] + i0, 1, np, YA[0] + i0, YA[1] + i0, np, 1,
                  [&](int b, int i, int j, WT v) {
                    if (i < kb && j < kb)
                      c.gb[b * K2 + i * K + j] = (double)c.G[b][(i0 + i) * np + i0 + j] + (double)v;
                  });
      __syncthreads();
    }
    if (wave == 0) {
      if (mA == 0) {
        for (int e = lane; e < kb * kb; e += 64) {
          int r = e / kb, cc = e - r * kb;
          c.gb[r * K + cc] = (double)c.G[0][(i0 + r) * np + i0 + cc];
          c.gb[K2 + r * K + cc] = (double)c.G[1][(i0 + r) * np + i0 + cc];
        }
      }
      decide_block(c, l, i0, kb, seed, sweep, fl, ldrun);
    }
    __syncthreads();
    clk.stop(c.st, PH_DECIDE);
    const int m = c.cnt[(i0 / K) & 1];
    acc_total += m;
    if (m > 0) {
      const int mp = (m + 3) & ~3;
      // ---- columns and rows of the true G at the accepted sites
      if (mA > 0) {
        const int mr = (mp + 15) & ~15;
        {
          // thread -> column t = tid % mr (mr = 16 or 32 divides NT), rows u = tid / mr + k NT / mr
          const int t = tid & (mr - 1), ustep = NT / mr;
          const int col = (t < m) ? i0 + c.site[t] : -1;
#pragma unroll
          for (int b = 0; b < 2; ++b)
            for (int u = tid / mr; u < mA; u += ustep) {
              Ys[b][u * K16 + t] = (col >= 0) ? YA[b][(size_t)u * np + col] : (WT)0;
              Xs[b][t * KT + u] = (col >= 0) ? XA[b][(size_t)u * np + col] : (WT)0;
            }
        }
        __syncthreads();
        wave_gemm<WT>(2, np, mr, mA, XA[0], XA[1], 1, np, Ys[0], Ys[1], K16, 1,
                     [&](int b, int i, int j, WT v) {
                       if (j < m)
                         Cc[b][(size_t)j * np + i] =
                             (WT)(((i < n) ? (double)c.G[b][i * np + i0 + c.site[j]] : 0.0) + (double)v);
                     });
        wave_gemm<WT>(2, mr, np, mA, Xs[0], Xs[1], KT, 1, YA[0], YA[1], np, 1,
                     [&](int b, int i, int j, WT v) {
                       if (i < m)
                         Rw[b][(size_t)i * np + j] =
                             (WT)(((j < n) ? (double)c.G[b][(i0 + c.site[i]) * np + j] : 0.0) + (double)v);
                     });
        __syncthreads();
      }
      // ---- the block's Sherman-Morrison vectors, appended to the panels at mA .. mA + mp
      for (int e = tid; e < 4 * np; e += NT) {
        const int kind = e / (2 * np);          // 0: X rows, 1: Y columns
        const int sp = (e / np) & 1;
        const int r = e - (e / np) * np;        // row (X) or column (Y)
        const WT* G0 = c.G[sp];
        const double* cf = sp ? c.cfd : c.cfu;
        const double* xbs = c.xb + sp * K2;
        const double* ybs = c.yb + sp * K2;
        double v[SM_KMAX];
#pragma unroll
        for (int t = 0; t < SM_KMAX; ++t) {
          v[t] = 0.0;
          if (t < m && r < n) {
            if (kind == 0)
              v[t] = mA ? (double)Cc[sp][(size_t)t * np + r] : (double)G0[r * np + i0 + c.site[t]];
            else
              v[t] = mA ? (double)Rw[sp][(size_t)t * np + r] : (double)G0[(i0 + c.site[t]) * np + r];
          }
        }
        if (kind == 0) sm_vec_x(m, c.site, cf, ybs, K, v);
        else sm_vec_y(m, r, i0, n, c.site, xbs, K, v);
        WT* P = (kind == 0 ? XA[sp] : YA[sp]) + (size_t)mA * np;
#pragma unroll
        for (int t = 0; t < SM_KMAX; ++t)
          if (t < mp) P[(size_t)t * np + r] = (t < m) ? (WT)v[t] : (WT)0;
      }
      __syncthreads();
      clk.stop(c.st, PH_PANEL);
      mA += mp;
    }
    // ---- G += XA YA when the next block might not fit, and at the end of the slice
    if (mA > 0 && (i0 + K >= n || mA + K > KT)) {
      wave_gemm_add<WT>(2, np, np, mA, XA[0], XA[1], 1, np, YA[0], YA[1], np, 1, c.G[0], c.G[1], np);
      __syncthreads();
      clk.stop(c.st, PH_FLUSH);
      mA = 0;
    }
  }
  if (tid == 0) {
    c.st->attempted += n;
    c.st->accepted += acc_total;
  }
}

// ------------------------------------------------------------------------------ stacks
// Pointers into the right stack (entry j: UDT of B(L, j*stab)^T) and the left factors.
template <typename WT>
__device__ __forceinline__ double* stkU(Ctx<WT>& c, int sp, int j) {
  const size_t nn = (size_t)c.np * c.np;
  return c.stack + ((size_t)sp * c.J + j) * (2 * nn + c.np);
}
template <typename WT>
__device__ __forceinline__ double* stkT(Ctx<WT>& c, int sp, int j) { return stkU(c, sp, j) + (size_t)c.np * c.np; }
template <typename WT>
__device__ __forceinline__ double* stkD(Ctx<WT>& c, int sp, int j) { return stkU(c, sp, j) + 2 * (size_t)c.np * c.np; }
template <typename WT>
__device__ __forceinline__ double* lftU(Ctx<WT>& c, int sp) {
  const size_t nn = (size_t)c.np * c.np;
  return c.left + (size_t)sp * (3 * nn + c.np);
}
template <typename WT>
__device__ __forceinline__ double* lftT(Ctx<WT>& c, int sp, int k) { return lftU(c, sp) + (size_t)(1 + k) * c.np * c.np; }
template <typename WT>
__device__ __forceinline__ double* lftD(Ctx<WT>& c, int sp) { return lftU(c, sp) + 3 * (size_t)c.np * c.np; }

// Left stack of the alternating sweeps: entry j = UDT of B(j*stab, 0), written by up sweeps.
template <typename WT>
__device__ __forceinline__ double* lstkU(Ctx<WT>& c, int sp, int j) {
  const size_t nn = (size_t)c.np * c.np;
  return c.lstack + ((size_t)sp * c.J + j) * (2 * nn + c.np);
}
template <typename WT>
__device__ __forceinline__ double* lstkT(Ctx<WT>& c, int sp, int j) { return lstkU(c, sp, j) + (size_t)c.np * c.np; }
template <typename WT>
__device__ __forceinline__ double* lstkD(Ctx<WT>& c, int sp, int j) { return lstkU(c, sp, j) + 2 * (size_t)c.np * c.np; }

// Equal-time estimators of the current G(l) (after every attempt of slice l, both directions),
// added to the chain's per-slice sums: double occupancy and kinetic energy per site as in
// measure_kernel.
template <typename WT>
__device__ __forceinline__ void slice_measure(Ctx<WT>& c) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np, tid = threadIdx.x;
  double docc = 0.0, kin = 0.0;
  for (int i = tid; i < n; i += NT) {
    const double gu = (double)c.G[0][i * np + i], gd = (double)c.G[1][i * np + i];
    docc += (1.0 - gu) * (1.0 - gd);
  }
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    const double t = a.Tm[i * np + j];
    if (t != 0.0)
      kin += t * (2.0 * (i == j ? 1.0 : 0.0) - (double)c.G[0][j * np + i] - (double)c.G[1][j * np + i]);
  }
  docc = wave_sum(docc);
  kin = wave_sum(kin);
  if ((tid & 63) == 0) {
    c.red.v[tid >> 6] = docc;
    c.red.v[NW + (tid >> 6)] = kin;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < NW; ++w) { s0 += c.red.v[w]; s1 += c.red.v[NW + w]; }
    c.st->slice_docc += s0 / n;
    c.st->slice_kin += s1 / n;
    c.st->slice_meas += 1;
  }
  __syncthreads();
}

// Build stack entries j = J-1 down to j_lo: entry j = UDT of B(L, j*stab)^T.
template <typename WT>
__device__ __forceinline__ void build_right(Ctx<WT>& c, int j_lo) {
  const KArgs& a = *c.a;
  for (int sp = 0; sp < 2; ++sp) {
    for (int j = c.J - 1; j >= j_lo; --j) {
      const int lo = j * c.stab, hi = min(c.L, (j + 1) * c.stab);
      const bool top = (j == c.J - 1);
      udt_push(c, sp, true, lo, hi, top ? a.eye : stkU(c, sp, j + 1), top ? a.ones : stkD(c, sp, j + 1),
               top ? a.eye : stkT(c, sp, j + 1), stkU(c, sp, j), stkD(c, sp, j), stkT(c, sp, j));
    }
  }
}

// Load the working G from the FP64 record.
template <typename WT>
__device__ __forceinline__ void load_green(Ctx<WT>& c) {
  const size_t nn = (size_t)c.np * c.np;
  for (size_t e = threadIdx.x; e < 2 * nn; e += NT) {
    int sp = (int)(e / nn);
    c.G[sp][e - sp * nn] = (WT)c.G64[e];
  }
  __syncthreads();
}

// ------------------------------------------------------------------------------ operations
template <typename WT>
__device__ __forceinline__ void op_init(Ctx<WT>& c, int idx) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np, L = c.L, tid = threadIdx.x;
  // fields: drawn from the seed or copied and validated
  const uint64_t seed = c.st->seed;
  for (int e = tid; e < L * np; e += NT) {
    int l = e / np, i = e - l * np;
    int8_t v = 0;
    if (i < n) {
      if (a.gen_fields) {
        const int ee = l * n + i;
        u64x4 w = philox4x64_10(u64x4{(uint64_t)(ee >> 2), 0ull, 0ull, 0ull}, seed, 0ull);
        uint64_t word = (ee & 3) == 0 ? w.x0 : (ee & 3) == 1 ? w.x1 : (ee & 3) == 2 ? w.x2 : w.x3;
        v = (word & 1ull) ? 1 : -1;
      } else {
        v = a.fields_in[((size_t)idx * L + l) * n + i];
        if (v != 1 && v != -1) { atomicOr(a.err, 1); v = 1; }
      }
    }
    c.f[e] = v;
  }
  __syncthreads();
  build_right(c, 0);
  double ld;
  for (int sp = 0; sp < 2; ++sp) {
    fresh_green(c, sp, a.eye, a.ones, a.eye, stkU(c, sp, 0), stkD(c, sp, 0), stkT(c, sp, 0),
                c.G64 + (size_t)sp * np * np, &ld, false);
    if (tid == 0) c.st->logdet[sp] = ld;
  }
  if (tid == 0) c.st->stack_ok = 1;
  __syncthreads();
}

// Fresh-G bookkeeping of one spin at a stabilisation point: drift, log-det error, flags.
template <typename WT>
__device__ __forceinline__ void stab_record(Ctx<WT>& c, int sp, double dr, double ld, double* ldrun) {
  const KArgs& a = *c.a;
  if (threadIdx.x == 0) {
    ChainStats* st = c.st;
    if (dr > st->max_drift || dr != dr) st->max_drift = dr;
    if (!(dr <= a.drift_limit)) st->flags |= FLAG_DRIFT;
    double e = fabs(ld - ldrun[sp]);
    if (e > st->max_logdet_err) st->max_logdet_err = e;
    ldrun[sp] = ld;
  }
  __syncthreads();
}

// n_sweeps sweeps.  Up sweep: wrap to G(l), attempt slice l, and at l = k stab and l = L push
// the chunk onto the left UDT and take the fresh G(l) from it and the right stack entry (built
// afresh at the start of the sweep, or left by the previous down sweep).  Down sweep (odd global
// sweeps of the alternating mode): attempt slice l at G(l), unwrap to G(l-1), and at
// l - 1 = k stab push the chunk onto the right UDT (into stack entry k) and take the fresh G from
// it and the left stack entry k written by the previous up sweep.
template <typename WT>
__device__ __forceinline__ void op_sweep(Ctx<WT>& c, int n_sweeps) {
  const KArgs& a = *c.a;
  const int np = c.np, L = c.L, tid = threadIdx.x;
  const bool alt = (a.sweep_mode & 1) && c.lstack;
  const bool per_slice = (a.sweep_mode & 2) != 0;
  load_green(c);
  PhaseClock clk, total;
  for (int s = 0; s < n_sweeps; ++s) {
    total.start();
    double* ldrun = c.misc;   // running log|det| per spin from accepted ratios
    const bool down = alt && (c.st->sweeps_done & 1);
    const bool stack_ok = c.st->stack_ok != 0;
    __syncthreads();
    if (tid == 0) { ldrun[0] = c.st->logdet[0]; ldrun[1] = c.st->logdet[1]; }
    __syncthreads();
    if (!down) {
      clk.start();
      if (!alt || !stack_ok) build_right(c, 1);
      clk.stop(c.st, PH_RIGHT);
      int cur = 0;     // which left T buffer is current
      int l_prev = 0;  // last stabilisation slice
      for (int l = 1; l <= L; ++l) {
        clk.start();
        wrap_both(c, l);
        clk.stop(c.st, PH_WRAP);
        if (c.stage && a.KT > 0) metropolis_slice2(c, l, ldrun);
        else metropolis_slice(c, l, ldrun);
        __syncthreads();
        if (per_slice) slice_measure(c);
        clk.start();
        if (l % c.stab == 0 || l == L) {
          const int jr = l / c.stab;   // stack entry at l (unused when l == L)
          const bool last = (l == L);
          for (int sp = 0; sp < 2; ++sp) {
            const bool first = (l_prev == 0);
            double *Ud, *dd, *Td;
            if (alt) {
              const int jp = l_prev / c.stab;
              Ud = last ? lftU(c, sp) : lstkU(c, sp, jr);
              dd = last ? lftD(c, sp) : lstkD(c, sp, jr);
              Td = last ? lftT(c, sp, 0) : lstkT(c, sp, jr);
              udt_push(c, sp, false, l_prev, l, first ? a.eye : lstkU(c, sp, jp),
                       first ? a.ones : lstkD(c, sp, jp), first ? a.eye : lstkT(c, sp, jp), Ud, dd, Td);
            } else {
              Ud = lftU(c, sp);
              dd = lftD(c, sp);
              Td = lftT(c, sp, cur ^ 1);
              udt_push(c, sp, false, l_prev, l, first ? a.eye : lftU(c, sp), first ? a.ones : lftD(c, sp),
                       first ? a.eye : lftT(c, sp, cur), Ud, dd, Td);
            }
            clk.stop(c.st, PH_LEFT);
            double ld;
            double dr = fresh_green(c, sp, Ud, dd, Td, last ? a.eye : stkU(c, sp, jr),
                                    last ? a.ones : stkD(c, sp, jr), last ? a.eye : stkT(c, sp, jr),
                                    last ? c.G64 + (size_t)sp * np * np : nullptr, &ld, true);
            stab_record(c, sp, dr, ld, ldrun);
            clk.stop(c.st, PH_FRESH);
          }
          cur ^= 1;
          l_prev = l;
        }
      }
      if (tid == 0) c.st->stack_ok = 0;   // the fields changed under the right stack
    } else {
      int r_prev = L;   // the right UDT covers B(L, r_prev)
      for (int l = L; l >= 1; --l) {
        if (c.stage && a.KT > 0) metropolis_slice2(c, l, ldrun);
        else metropolis_slice(c, l, ldrun);
        __syncthreads();
        if (per_slice) slice_measure(c);
        clk.start();
        unwrap_both(c, l);
        clk.stop(c.st, PH_WRAP);
        if ((l - 1) % c.stab == 0) {
          const int j = (l - 1) / c.stab;
          const bool top = (r_prev == L);
          const int jp = r_prev / c.stab;
          for (int sp = 0; sp < 2; ++sp) {
            udt_push(c, sp, true, l - 1, r_prev, top ? a.eye : stkU(c, sp, jp),
                     top ? a.ones : stkD(c, sp, jp), top ? a.eye : stkT(c, sp, jp), stkU(c, sp, j),
                     stkD(c, sp, j), stkT(c, sp, j));
            clk.stop(c.st, PH_RIGHT);
            double ld;
            const bool bottom = (j == 0);
            double dr = fresh_green(c, sp, bottom ? a.eye : lstkU(c, sp, j), bottom ? a.ones : lstkD(c, sp, j),
                                    bottom ? a.eye : lstkT(c, sp, j), stkU(c, sp, j), stkD(c, sp, j),
                                    stkT(c, sp, j), bottom ? c.G64 + (size_t)sp * np * np : nullptr, &ld, true);
            stab_record(c, sp, dr, ld, ldrun);
            clk.stop(c.st, PH_FRESH);
          }
          r_prev = l - 1;
        }
      }
      if (tid == 0) c.st->stack_ok = 1;   // entries 0 .. J-1 now describe the current fields
    }
    if (tid == 0) {
      c.st->logdet[0] = ldrun[0];
      c.st->logdet[1] = ldrun[1];
      c.st->sweeps_done += 1;
    }
    __syncthreads();
    total.stop(c.st, PH_SWEEP);
  }
}

// Fresh G(slice) of the current field from scratch (left chain from slice 1, right chain from
// slice L, both chunked by stab), into the working G of both spins.
template <typename WT>
__device__ __forceinline__ void fresh_at(Ctx<WT>& c, int slice) {
  if (threadIdx.x == 0) c.st->stack_ok = 0;   // stack entries 0 and 1 serve as scratch below
  const KArgs& a = *c.a;
  const int L = c.L;
  for (int sp = 0; sp < 2; ++sp) {
    // left: B(slice, 0) into the left buffers (T ping-pong)
    int cur = 0;
    bool have = false;
    for (int lo = 0; lo < slice; lo += c.stab) {
      const int hi = min(slice, lo + c.stab);
      udt_push(c, sp, false, lo, hi, have ? lftU(c, sp) : a.eye, have ? lftD(c, sp) : a.ones,
               have ? lftT(c, sp, cur) : a.eye, lftU(c, sp), lftD(c, sp), lftT(c, sp, cur ^ 1));
      cur ^= 1;
      have = true;
    }
    // right: B(L, slice)^T into stack slot 0 (T ping-pong through slot 1's T when J > 1)
    bool rhave = false;
    int rcur = 0;
    double* rT[2] = {stkT(c, sp, 0), c.J > 1 ? stkT(c, sp, 1) : stkT(c, sp, 0)};
    for (int hi = L; hi > slice; hi -= c.stab) {
      const int lo = max(slice, hi - c.stab);
      udt_push(c, sp, true, lo, hi, rhave ? stkU(c, sp, 0) : a.eye, rhave ? stkD(c, sp, 0) : a.ones,
               rhave ? rT[rcur] : a.eye, stkU(c, sp, 0), stkD(c, sp, 0), rT[rcur ^ 1]);
      rcur ^= 1;
      rhave = true;
    }
    double ld;
    fresh_green(c, sp, have ? lftU(c, sp) : a.eye, have ? lftD(c, sp) : a.ones,
                have ? lftT(c, sp, cur) : a.eye, rhave ? stkU(c, sp, 0) : a.eye,
                rhave ? stkD(c, sp, 0) : a.ones, rhave ? rT[rcur] : a.eye, nullptr, &ld, false);
  }
}

template <typename WT>
__device__ __forceinline__ void op_debug_green(Ctx<WT>& c, int chain) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np;
  fresh_at(c, a.slice);
  for (int w = 1; w <= a.n_wraps; ++w) wrap_both(c, a.slice + w);
  for (int w = 0; w < -a.n_wraps; ++w) unwrap_both(c, a.slice - w);
  double* out = a.out + (size_t)chain * 2 * n * n;
  for (int e = threadIdx.x; e < 2 * n * n; e += NT) {
    int sp = e / (n * n), r = (e / n) % n, col = e % n;
    out[e] = (double)c.G[sp][r * np + col];
  }
}

template <typename WT>
__device__ __forceinline__ void op_debug_ratios(Ctx<WT>& c, int chain) {
  const KArgs& a = *c.a;
  const int n = c.n, np = c.np;
  fresh_at(c, a.slice);
  const int8_t* fl = c.f + (size_t)(a.slice - 1) * np;
  double* out = a.out + (size_t)chain * 2 * n;
  for (int e = threadIdx.x; e < 2 * n; e += NT) {
    int sp = e / n, i = e % n;
    int s = fl[i];
    double d = sp ? a.ddn[s > 0] : a.dup[s > 0];
    out[e] = 1.0 + d * (1.0 - (double)c.G[sp][i * np + i]);
  }
}

}  // namespace dqmc
