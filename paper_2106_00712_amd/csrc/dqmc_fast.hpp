// Fast sweep path for chains with N <= 64 sites (padded size NP in {16, 32, 64}).
//
// Same method and decisions as the generic path (dqmc_device.hpp), organised for latency:
//   * the Green's functions of both spins stay in LDS; at a stabilisation point they are
//     parked in the chain's workspace so that the whole 4*NP*NP-double LDS arena serves the
//     QR and Gauss-Jordan work of both spins at once;
//   * column-pivoted Householder QR and Gauss-Jordan inversion run one wavefront per spin with
//     the matrix in registers (dqmc_stab.hpp): no workgroup barrier inside a factorisation;
//   * the wavefront that decides a block of K sites keeps the K x K block of both spins in
//     registers and moves rows and columns between lanes with cross-lane permutes;
//   * the MFMA operand fragments of e^{-dtau T} (rows) and e^{+dtau T} (columns) that a
//     wavefront needs are loaded once per launch and kept in registers.
#pragma once
#include "dqmc_device.hpp"
#include "dqmc_stab.hpp"

namespace dqmc {
namespace fast {

template <typename T> __device__ __forceinline__ T bcast(T v, int lane);
template <> __device__ __forceinline__ double bcast<double>(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
template <> __device__ __forceinline__ int bcast<int>(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

// Largest key over the 64 lanes (ties -> smallest index; idx < 0 = no candidate).
__device__ __forceinline__ void wave_argmax(double& key, int& idx) {
  if (idx < 0) key = -1.0;
  for (int o = 32; o > 0; o >>= 1) {
    double k2 = __shfl_xor(key, o);
    int i2 = __shfl_xor(idx, o);
    bool take = (i2 >= 0) && (idx < 0 || k2 > key || (k2 == key && i2 < idx));
    if (take) { key = k2; idx = i2; }
  }
}

template <int NP_, typename WT, int KB_>
struct Fast {
  static constexpr int NP = NP_;
  static constexpr int KB = KB_;                 // sites per delayed-update block
  static constexpr int NN = NP * NP;
  static constexpr int TBK = NP / 16;             // 16-blocks per dimension
  static constexpr int KS = NP / 4;               // MFMA k-steps over NP
  static constexpr int UNITS = 2 * TBK;           // (spin, row-or-column block) units of a wrap GEMM
  static constexpr int UPW = (UNITS + NW - 1) / NW;   // units per wave
  static constexpr int RPL = KB * KB / 32;        // block rows per lane in the decide phase
  static constexpr int GSLOTS = sizeof(WT) == 8 ? 2 : 1;   // NN-double slots the G pair occupies
  typedef typename acc4<WT>::type accw;

  // LDS: arena of 4 NN doubles, then the vectors below.
  struct Lds {
    double* arena;
    double *xb, *yb;       // [2][KB][KB] block records: x_t (column t), y_t (row t)
    double *cf;            // [2][KB]
    int *site, *cnt;       // [KB], [4]
    double *vd, *bt, *dd, *sgn;  // per spin [2][NP]
    int *rank, *ordv;      // per spin [2][NP]
    double* misc;          // [16]
    double* red;           // [2*NW]
  };
  static __host__ __device__ size_t lds_bytes() {
    return (4 * (size_t)NN + 4 * KB * KB + 2 * KB + 4 * 2 * NP + 16 + 2 * NW) * sizeof(double) +
           (KB + 4 + 4 * NP) * sizeof(int) + 64;
  }
  static __device__ Lds carve(double* lds) {
    Lds L;
    double* p = lds;
    L.arena = p; p += 4 * NN;
    L.xb = p; p += 2 * KB * KB;
    L.yb = p; p += 2 * KB * KB;
    L.cf = p; p += 2 * KB;
    L.vd = p; p += 2 * NP;
    L.bt = p; p += 2 * NP;
    L.dd = p; p += 2 * NP;
    L.sgn = p; p += 2 * NP;
    L.misc = p; p += 16;
    L.red = p; p += 2 * NW;
    int* ip = (int*)p;
    L.site = ip; ip += KB;
    L.cnt = ip; ip += 4;
    L.rank = ip; ip += 2 * NP;
    L.ordv = ip; ip += 2 * NP;
    return L;
  }
  static __device__ __forceinline__ double* slot(const Lds& L, int k) { return L.arena + (size_t)k * NN; }
  static __device__ __forceinline__ WT* gptr(const Lds& L, int sp) { return (WT*)L.arena + (size_t)sp * NN; }
  static __device__ __forceinline__ WT* wptr(const Lds& L, int k) { return (WT*)(L.arena + (size_t)(GSLOTS + k) * NN); }

  // ------------------------------------------------------------------ register-cached operands
  // A wrap GEMM is split in UNITS = 2 spins x TBK blocks; wave w owns units w and w + NW; unit u
  // is (spin u / TBK, block u % TBK).  For NP <= 64 every unit of a wave has the same block
  // (w % TBK), so one set of fragments per wave covers both spins.
  static constexpr bool F32 = sizeof(WT) == 4;
  struct Regs {
    double kA[KS];                 // e^{-dtau T}: rows of the wave's block (A fragments), FP64
    WT kBw[KS];                    // e^{+dtau T}: columns of the wave's block (B fragments)
    float kA32[F32 ? KS : 1];      // e^{-dtau T} rows in FP32 (FP32-wrap precision only)
  };
  static __device__ __forceinline__ void load_regs(const KArgs& a, Regs& R) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const WT* Kiw = kexpinv<WT>(a);
    const int blk = wave % TBK;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      R.kA[s] = a.expK[(blk * 16 + li) * NP + 4 * s + lk];
      R.kBw[s] = Kiw[(4 * s + lk) * NP + blk * 16 + li];
      if constexpr (F32) R.kA32[s] = a.expK32[(blk * 16 + li) * NP + 4 * s + lk];
    }
  }

  // C_sp = e^{-dtau T} X_sp for both spins (X in LDS, row-major NP x NP, element type T);
  // epi(sp, i, j, v) per output element.  Uses the cached A fragments.
  template <typename T, typename Epi>
  static __device__ __forceinline__ void gemm_k_left(const T (&kA)[KS], const T* X0, const T* X1, Epi epi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int q = 0; q < UPW; ++q) {
      const int u = wave + q * NW;
      if (u >= UNITS) break;
      const int sp = u / TBK, ti = u % TBK;
      const T* X = sp ? X1 : X0;
#pragma unroll
      for (int tj = 0; tj < TBK; ++tj) {
        typename acc4<T>::type acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = mfma(kA[s], X[(4 * s + lk) * NP + tj * 16 + li], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) epi(sp, ti * 16 + out_row<T>(v, lane), tj * 16 + li, acc[v]);
      }
    }
  }

  // C_sp = Y_sp e^{+dtau T} for both spins (Y in LDS, row-major), cached B fragments; the unit's
  // block is a column block.
  template <typename Epi>
  static __device__ __forceinline__ void gemm_kinv_right(const WT (&kB)[KS], const WT* Y0, const WT* Y1, Epi epi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int q = 0; q < UPW; ++q) {
      const int u = wave + q * NW;
      if (u >= UNITS) break;
      const int sp = u / TBK, tj = u % TBK;
      const WT* Y = sp ? Y1 : Y0;
#pragma unroll
      for (int ti = 0; ti < TBK; ++ti) {
        accw acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = mfma(Y[(ti * 16 + li) * NP + 4 * s + lk], kB[s], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) epi(sp, ti * 16 + out_row<WT>(v, lane), tj * 16 + li, acc[v]);
      }
    }
  }

  // Generic NP x NP x K products for both spins, operands anywhere (strided), tiles dealt to
  // the waves round-robin.
  template <typename T, typename Epi>
  static __device__ __forceinline__ void gemm2(int K, const T* A0, const T* A1, int sai, int sak,
                                               const T* B0, const T* B1, int sbk, int sbj, Epi epi) {
    wg_gemm<T>(2, NP, NP, K, A0, A1, sai, sak, B0, B1, sbk, sbj, epi);
  }

  // ------------------------------------------------------------------ the sweep
  struct Chain {
    const KArgs* a;
    ChainStats* st;
    int8_t* f;
    double* G64;
    WT* Gsave;       // [2][NN] parking place of the working G (workspace)
    double* stack;
    double* left;
    int n, L, stab, J;
  };
  static __device__ __forceinline__ double* stkU(const Chain& c, int sp, int j) {
    return c.stack + ((size_t)sp * c.J + j) * (2 * (size_t)NN + NP);
  }
  static __device__ __forceinline__ double* stkT(const Chain& c, int sp, int j) { return stkU(c, sp, j) + NN; }
  static __device__ __forceinline__ double* stkD(const Chain& c, int sp, int j) { return stkU(c, sp, j) + 2 * NN; }
  static __device__ __forceinline__ double* lftU(const Chain& c, int sp) { return c.left + (size_t)sp * (3 * (size_t)NN + NP); }
  static __device__ __forceinline__ double* lftT(const Chain& c, int sp, int k) { return lftU(c, sp) + (size_t)(1 + k) * NN; }
  static __device__ __forceinline__ double* lftD(const Chain& c, int sp) { return lftU(c, sp) + 3 * (size_t)NN; }

  static __device__ void park_green(const Chain& c, const Lds& L) {
    for (int e = threadIdx.x; e < 2 * NN; e += NT) c.Gsave[e] = ((WT*)L.arena)[e];
  }
  static __device__ void unpark_green(const Chain& c, const Lds& L) {
    for (int e = threadIdx.x; e < 2 * NN; e += NT) ((WT*)L.arena)[e] = c.Gsave[e];
  }

  // Multiply a chunk of slices onto U Diag(d) for both spins and factorise (UDT), exactly as the
  // generic udt_push: left chunks B_hi ... B_lo+1 U D, right chunks (transposed world)
  // B_lo+1^T ... B_hi^T U D with B_l^T = e^{-dtau T} V_l (e^{-dtau T} is symmetric).
  // The arena must be free (G parked).  Results: Ud, dd, Td per spin (global).
  static __device__ void push_both(const Chain& c, const Lds& L, const Regs& R, bool right, int lo, int hi,
                                   const double* const Us[2], const double* const ds[2],
                                   const double* const Ts[2], double* const Ud[2], double* const Dd[2],
                                   double* const Td[2]) {
    const KArgs& a = *c.a;
    const int n = c.n;
    int cur = 2, nxt = 0;   // slot pair (cur + sp), (nxt + sp)
    {
      const int8_t* fh = c.f + (size_t)(hi - 1) * NP;
      for (int e = threadIdx.x; e < 2 * NN; e += NT) {
        const int sp = e / NN, ee = e - sp * NN, i = ee / NP, j = ee - i * NP;
        double v = Us[sp][ee] * ds[sp][j];
        if (right) v *= (i < n) ? vfac(a, sp, fh[i]) : 1.0;
        slot(L, cur + sp)[ee] = v;
      }
    }
    __syncthreads();
    PhaseClock pc;
    pc.start();
    const int steps = hi - lo;
    for (int t = 0; t < steps; ++t) {
      // left: slice lo+1+t, scale rows after the product; right: slice hi-t, the next slice's
      // scale (hi-t-1) after the product unless this is the last factor
      const int lsc = right ? (hi - t - 1) : (lo + 1 + t);
      const bool scale = right ? (lsc >= lo + 1) : true;
      const int8_t* fs = c.f + (size_t)(scale ? lsc - 1 : 0) * NP;
      double* o0 = slot(L, nxt);
      double* o1 = slot(L, nxt + 1);
      gemm_k_left<double>(R.kA, slot(L, cur), slot(L, cur + 1), [&](int sp, int i, int j, double v) {
        double s = (scale && i < n) ? vfac(a, sp, fs[i]) : 1.0;
        (sp ? o1 : o0)[i * NP + j] = s * v;
      });
      __syncthreads();
      int tmp = cur; cur = nxt; nxt = tmp;
    }
    pc.stop(c.st, PH_CHUNK);
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {
      const int sp = wave;
      PhaseClock qc;
      qc.start();
      DQMC_LDS double* X = (DQMC_LDS double*)slot(L, cur + sp);
      DQMC_LDS double* vd = (DQMC_LDS double*)(L.vd + sp * NP);
      DQMC_LDS double* bt = (DQMC_LDS double*)(L.bt + sp * NP);
      DQMC_LDS double* dd = (DQMC_LDS double*)(L.dd + sp * NP);
      DQMC_LDS double* sg = (DQMC_LDS double*)(L.sgn + sp * NP);
      DQMC_LDS int* rk = (DQMC_LDS int*)(L.rank + sp * NP);
      DQMC_LDS int* ov = (DQMC_LDS int*)(L.ordv + sp * NP);
      DQMC_LDS double* Vb = (DQMC_LDS double*)slot(L, nxt + sp);
      stab::qr_factor<NP>(n, X, Vb, vd, bt, rk, ov, dd, sg, &c.st->flags);
      qc.stop(c.st, PH_QR);
      stab::qr_form_q<NP>(n, Vb, vd, bt, sg, Ud[sp]);
      qc.stop(c.st, PH_QFORM);
      // d to the workspace; T' = D^{-1} S R P^T in place (column c of R lives in lane c)
      const int cc = threadIdx.x & 63;
      if (cc < NP) {
        Dd[sp][cc] = (cc < n) ? dd[cc] : 1.0;
        const int rkc = (cc < n) ? rk[cc] : -1;
        for (int aa = 0; aa < NP; ++aa) {
          double v = 0.0;
          if (aa < n && rkc >= aa) v = sg[aa] * X[aa * NP + cc] / dd[aa];
          X[aa * NP + cc] = v;
        }
      }
      wave_sync();
    }
    __syncthreads();
    pc.start();
    gemm2<double>(NP, slot(L, cur), slot(L, cur + 1), NP, 1, Ts[0], Ts[1], NP, 1,
                  [&](int sp, int i, int j, double v) { Td[sp][i * NP + j] = v; });
    __syncthreads();
    pc.stop(c.st, PH_TMUL);
  }

  // Right stack entries j = J-1 .. 1 for both spins (G parked around it).
  static __device__ void build_right(const Chain& c, const Lds& L, const Regs& R) {
    const KArgs& a = *c.a;
    for (int j = c.J - 1; j >= 1; --j) {
      const int lo = j * c.stab, hi = min(c.L, (j + 1) * c.stab);
      const bool top = (j == c.J - 1);
      const double* Us[2] = {top ? a.eye : stkU(c, 0, j + 1), top ? a.eye : stkU(c, 1, j + 1)};
      const double* ds[2] = {top ? a.ones : stkD(c, 0, j + 1), top ? a.ones : stkD(c, 1, j + 1)};
      const double* Ts[2] = {top ? a.eye : stkT(c, 0, j + 1), top ? a.eye : stkT(c, 1, j + 1)};
      double* Ud[2] = {stkU(c, 0, j), stkU(c, 1, j)};
      double* Dd[2] = {stkD(c, 0, j), stkD(c, 1, j)};
      double* Td[2] = {stkT(c, 0, j), stkT(c, 1, j)};
      push_both(c, L, R, true, lo, hi, Us, ds, Ts, Ud, Dd, Td);
    }
  }

  // Fresh G of both spins from the left factors and the right factors (two-sided split at 1),
  // into the LDS G; drift against the parked G; optional FP64 record.  Arena free on entry.
  static __device__ void fresh_both(const Chain& c, const Lds& L, const double* const UL[2],
                                    const double* const dL[2], const double* const TL[2],
                                    const double* const UR[2], const double* const dR[2],
                                    const double* const TR[2], bool record, double* drift,
                                    double* logdet) {
    const int n = c.n, tid = threadIdx.x;
    // slots: M (2 + sp), M^{-1} (sp), then Z' = M^{-1} DLb^{-1} UL^T DRb^{-1}-rows back in (2 + sp)
    double* iLb = L.vd;   // [2][NP]
    double* iRb = L.bt;
    PhaseClock pc;
    pc.start();
    for (int e = tid; e < 2 * NP; e += NT) {
      const int sp = e / NP, i = e - sp * NP;
      iLb[e] = 1.0 / fmax(dL[sp][i], 1.0);
      iRb[e] = 1.0 / fmax(dR[sp][i], 1.0);
    }
    __syncthreads();
    // M = DLb^{-1} (UL^T UR) DRb^{-1} + DLs (TL TR^T) DRs, accumulated in one pass per tile
    gemm2<double>(NP, UL[0], UL[1], 1, NP, UR[0], UR[1], NP, 1, [&](int sp, int i, int j, double v) {
      slot(L, 2 + sp)[i * NP + j] = v * iLb[sp * NP + i] * iRb[sp * NP + j];
    });
    __syncthreads();
    gemm2<double>(NP, TL[0], TL[1], NP, 1, TR[0], TR[1], 1, NP, [&](int sp, int i, int j, double v) {
      slot(L, 2 + sp)[i * NP + j] += fmin(dL[sp][i], 1.0) * v * fmin(dR[sp][j], 1.0);
    });
    __syncthreads();
    pc.stop(c.st, PH_FGEMM);
    const int wave = tid >> 6;
    if (wave < 2) {
      const int sp = wave;
      double la = stab::gj_inverse<NP>(n, (const DQMC_LDS double*)slot(L, 2 + sp),
                                       (DQMC_LDS double*)slot(L, sp),
                                       (const DQMC_LDS double*)(iLb + sp * NP),
                                       (DQMC_LDS int*)(L.ordv + sp * NP),
                                       (DQMC_LDS double*)(L.dd + sp * NP), &c.st->flags);
      if ((tid & 63) == 0) L.misc[8 + sp] = la;
    }
    __syncthreads();
    pc.stop(c.st, PH_GJ);
    // Z' = DRb^{-1} (M^{-1} DLb^{-1}) UL^T into the M slots
    gemm2<double>(NP, slot(L, 0), slot(L, 1), NP, 1, UL[0], UL[1], 1, NP,
                  [&](int sp, int i, int j, double v) { slot(L, 2 + sp)[i * NP + j] = v * iRb[sp * NP + i]; });
    __syncthreads();
    double dmax = 0.0;
    bool bad = false;
    gemm2<double>(NP, UR[0], UR[1], NP, 1, slot(L, 2), slot(L, 3), NP, 1, [&](int sp, int i, int j, double v) {
      const int e = i * NP + j;
      const WT* Go = c.Gsave + (size_t)sp * NN;
      dmax = fmax(dmax, fabs((double)Go[e] - v));
      if (!(fabs(v) < 1e300)) bad = true;
      gptr(L, sp)[e] = (WT)v;
      if (record) c.G64[(size_t)sp * NN + e] = v;
    });
    __syncthreads();
    pc.stop(c.st, PH_GOUT);
    if (bad) atomicOr(&c.st->flags, FLAG_NONFINITE);
    // log|det| per spin: sum log dLb + sum log dRb + log|det M|
    double part[2] = {0.0, 0.0};
    for (int i = tid; i < n; i += NT) {
      part[0] += log(fmax(dL[0][i], 1.0)) + log(fmax(dR[0][i], 1.0));
      part[1] += log(fmax(dL[1][i], 1.0)) + log(fmax(dR[1][i], 1.0));
    }
    part[0] = wave_sum(part[0]);
    part[1] = wave_sum(part[1]);
    dmax = wave_max(dmax);
    if ((tid & 63) == 0) {
      L.red[(tid >> 6)] = part[0];
      L.red[NW + (tid >> 6)] = part[1];
      L.misc[12 + (tid >> 6)] = dmax;
    }
    __syncthreads();
    double l0 = L.misc[8], l1 = L.misc[9], dm = 0.0;
    for (int w = 0; w < NW; ++w) { l0 += L.red[w]; l1 += L.red[NW + w]; dm = fmax(dm, L.misc[12 + w]); }
    logdet[0] = l0;
    logdet[1] = l1;
    *drift = dm;
    __syncthreads();
  }

  // Wrap both spins: G <- V_l e^{-dtau T} G e^{+dtau T} V_l^{-1}.
  static __device__ void wrap(const Chain& c, const Lds& L, const Regs& R, int l) {
    const KArgs& a = *c.a;
    const int n = c.n;
    const int8_t* fl = c.f + (size_t)(l - 1) * NP;
    double* sr = L.vd;
    double* sc = L.bt;
    for (int e = threadIdx.x; e < 2 * NP; e += NT) {
      const int sp = e / NP, i = e - sp * NP;
      sr[e] = (i < n) ? vfac(a, sp, fl[i]) : 1.0;
      sc[e] = (i < n) ? vfac(a, sp, -fl[i]) : 1.0;
    }
    WT* T0 = wptr(L, 0);
    WT* T1 = T0 + NN;
    auto epi1 = [&](int sp, int i, int j, WT v) { (sp ? T1 : T0)[i * NP + j] = v; };
    if constexpr (F32) gemm_k_left<float>(R.kA32, (const float*)gptr(L, 0), (const float*)gptr(L, 1), epi1);
    else gemm_k_left<double>(R.kA, (const double*)gptr(L, 0), (const double*)gptr(L, 1), epi1);
    __syncthreads();
    gemm_kinv_right(R.kBw, T0, T1, [&](int sp, int i, int j, WT v) {
      gptr(L, sp)[i * NP + j] = (WT)(sr[sp * NP + i] * (double)v * sc[sp * NP + j]);
    });
    __syncthreads();
  }

  // Metropolis over the sites of slice l (see metropolis_slice in the generic path for the
  // derivation); blocks of KB sites decided by wave 0 with the block in registers.
  static __device__ void metropolis(const Chain& c, const Lds& L, int l, double* ldrun) {
    const KArgs& a = *c.a;
    const int n = c.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int8_t* fl = c.f + (size_t)(l - 1) * NP;
    const uint64_t seed = c.st->seed;
    const int64_t sweep = c.st->sweeps_done;
    double u_lane = 0.0;
    int s_lane = 0;
    if (wave == 0 && lane < n) {
      u_lane = accept_uniform(seed, sweep, l - 1, lane);
      s_lane = fl[lane];
    }
    int64_t acc_total = 0;
    PhaseClock clk;
    clk.start();
    WT* G0 = gptr(L, 0);
    WT* G1 = gptr(L, 1);
    for (int i0 = 0; i0 < n; i0 += KB) {
      const int kb = min(KB, n - i0);
      // the block's accept count alternates between two LDS words: after a block with no
      // accepts no barrier separates the other waves' read of its count from wave 0's write of
      // the next block's, so that write must not land on the word still being read
      const int par = (i0 / KB) & 1;
      if (wave == 0) {
        const int sp = lane >> 5, q = lane & 31, cc = q % KB, h = q / KB;
        const WT* Gs = sp ? G1 : G0;
        double gb[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int r = h * RPL + k;
          gb[k] = (r < kb && cc < kb) ? (double)Gs[(i0 + r) * NP + i0 + cc] : 0.0;
        }
        int m = 0;
        double ldu = 1.0, ldd = 1.0;   // products of accepted ratios (one log per block)
        int flg = 0;
        int64_t ties = 0;
        double* xb = L.xb + sp * KB * KB;
        double* yb = L.yb + sp * KB * KB;
#pragma unroll
        for (int ii = 0; ii < KB; ++ii) {
          if (ii < kb) {
            const int site = i0 + ii;
            const double u = bcast(u_lane, site);
            const int s = bcast(s_lane, site);
            const int ld = (ii / RPL) * KB + ii;
            const double gu = bcast(gb[ii % RPL], ld);
            const double gd = bcast(gb[ii % RPL], 32 + ld);
            const double du = a.dup[s > 0], dd = a.ddn[s > 0];
            const double ru = 1.0 + du * (1.0 - gu), rd = 1.0 + dd * (1.0 - gd);
            const double Rt = ru * rd;
            bool ok = true;
            if (!(fabs(Rt) < 1e300)) { flg |= FLAG_NONFINITE; ok = false; }
            else if (Rt < 0.0) { flg |= FLAG_NEGATIVE; ok = false; }
            if (ok && fabs(u - Rt) < 1e-9) ++ties;
            if (ok && u < Rt) {
              const double cu = du / ru, cd = dd / rd;
              const double cfs = sp ? cd : cu;
              double colv[RPL];
#pragma unroll
              for (int k = 0; k < RPL; ++k) colv[k] = __shfl(gb[k], sp * 32 + h * KB + ii);
              const double rowv = __shfl(gb[ii % RPL], sp * 32 + (ii / RPL) * KB + cc);
              const double y = ((cc == ii) ? 1.0 : 0.0) - rowv;
#pragma unroll
              for (int k = 0; k < RPL; ++k) {
                const double x = -cfs * colv[k];
                gb[k] += x * y;
                if (cc == 0) xb[(h * RPL + k) * KB + m] = x;
              }
              if (h == 0) yb[m * KB + cc] = y;
              if (lane == 0) {
                L.site[m] = ii;
                L.cf[m] = cu;
                L.cf[KB + m] = cd;
                fl[site] = (int8_t)(-s);
              }
              ldu *= fabs(ru);
              ldd *= fabs(rd);
              ++m;
            }
          }
        }
        if (lane == 0) {
          L.cnt[par] = m;
          ldrun[0] += log(ldu);
          ldrun[1] += log(ldd);
          if (flg) atomicOr(&c.st->flags, flg);
          c.st->near_ties += ties;
        }
      }
      __syncthreads();
      clk.stop(c.st, PH_DECIDE);
      const int m = L.cnt[par];
      acc_total += m;
      if (m == 0) continue;
      const int mp = (m + 3) & ~3;
      WT* X0 = wptr(L, 0);
      WT* Y0 = X0 + NP * KB;
      WT* X1 = X0 + 2 * NP * KB;
      WT* Y1 = X0 + 3 * NP * KB;
      // panels, one row of X or one column of Y per thread with the m terms in registers:
      //   x_t = -c_t (G[:, a_t] + sum_{t'<t} x_t' y_t'[a_t]),  y_t = e_{a_t} - G[a_t, :] - sum_{t'<t} x_t'[a_t] y_t'
      for (int e = tid; e < 4 * NP; e += NT) {
        const int kind = e / (2 * NP), sp = (e / NP) & 1, r = e % NP;
        const WT* Gs = sp ? G1 : G0;
        const double* xbs = L.xb + sp * KB * KB;
        const double* ybs = L.yb + sp * KB * KB;
        int at[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) at[t] = (t < m) ? L.site[t] : 0;
        double v[KB];
        if (kind == 0) {
#pragma unroll
          for (int t = 0; t < KB; ++t) {
            v[t] = 0.0;
            if (t < m) {
              double acc = (double)Gs[r * NP + i0 + at[t]];
#pragma unroll
              for (int t2 = 0; t2 < t; ++t2) acc += v[t2] * ybs[t2 * KB + at[t]];
              v[t] = -L.cf[sp * KB + t] * acc;
            }
          }
          WT* X = sp ? X1 : X0;
#pragma unroll
          for (int t = 0; t < KB; ++t)
            if (t < mp) X[t * NP + r] = (WT)v[t];
        } else {
#pragma unroll
          for (int t = 0; t < KB; ++t) {
            v[t] = 0.0;
            if (t < m) {
              const int ia = i0 + at[t];
              double acc = ((r == ia && r < n) ? 1.0 : 0.0) - (double)Gs[ia * NP + r];
#pragma unroll
              for (int t2 = 0; t2 < t; ++t2) acc -= xbs[at[t] * KB + t2] * v[t2];
              v[t] = acc;
            }
          }
          WT* Y = sp ? Y1 : Y0;
#pragma unroll
          for (int t = 0; t < KB; ++t)
            if (t < mp) Y[t * NP + r] = (WT)v[t];
        }
      }
      __syncthreads();
      clk.stop(c.st, PH_PANEL);
      wg_gemm<WT>(2, NP, NP, mp, X0, X1, 1, NP, Y0, Y1, NP, 1,
                  [&](int b, int i, int j, WT v) { (b ? G1 : G0)[i * NP + j] += v; });
      __syncthreads();
      clk.stop(c.st, PH_FLUSH);
    }
    if (tid == 0) {
      c.st->attempted += n;
      c.st->accepted += acc_total;
    }
  }

  static __device__ void run(const KArgs& a, int chain, int n_sweeps, double* lds) {
    const int tid = threadIdx.x;
    Lds L = carve(lds);
    Regs R;
    load_regs(a, R);
    char* cb = a.base + (size_t)chain * a.stride;
    Chain c;
    c.a = &a;
    c.st = (ChainStats*)(cb + a.o_stats);
    c.f = (int8_t*)(cb + a.o_fields);
    c.G64 = (double*)(cb + a.o_G64);
    c.Gsave = (WT*)(cb + a.o_Gw);
    c.stack = (double*)(cb + a.o_stack);
    c.left = (double*)(cb + a.o_left);
    c.n = a.n; c.L = a.L; c.stab = a.stab; c.J = a.J;
    for (int e = tid; e < 2 * NN; e += NT) ((WT*)L.arena)[e] = (WT)c.G64[e];
    __syncthreads();
    PhaseClock clk, total;
    for (int s = 0; s < n_sweeps; ++s) {
      total.start();
      clk.start();
      park_green(c, L);
      __syncthreads();
      build_right(c, L, R);
      unpark_green(c, L);
      __syncthreads();
      clk.stop(c.st, PH_RIGHT);
      double* ldrun = L.misc;
      if (tid == 0) { ldrun[0] = c.st->logdet[0]; ldrun[1] = c.st->logdet[1]; }
      __syncthreads();
      int cur = 0, l_prev = 0;
      for (int l = 1; l <= c.L; ++l) {
        clk.start();
        wrap(c, L, R, l);
        clk.stop(c.st, PH_WRAP);
        metropolis(c, L, l, ldrun);
        __syncthreads();
        clk.start();
        if (l % c.stab == 0 || l == c.L) {
          PhaseClock pk;
          pk.start();
          park_green(c, L);
          __syncthreads();
          pk.stop(c.st, PH_PARK);
          const bool first = (l_prev == 0);
          const double* Us[2] = {first ? a.eye : lftU(c, 0), first ? a.eye : lftU(c, 1)};
          const double* ds[2] = {first ? a.ones : lftD(c, 0), first ? a.ones : lftD(c, 1)};
          const double* Ts[2] = {first ? a.eye : lftT(c, 0, cur), first ? a.eye : lftT(c, 1, cur)};
          double* Ud[2] = {lftU(c, 0), lftU(c, 1)};
          double* Dd[2] = {lftD(c, 0), lftD(c, 1)};
          double* Td[2] = {lftT(c, 0, cur ^ 1), lftT(c, 1, cur ^ 1)};
          push_both(c, L, R, false, l_prev, l, Us, ds, Ts, Ud, Dd, Td);
          clk.stop(c.st, PH_LEFT);
          const bool last = (l == c.L);
          const int jr = l / c.stab;
          const double* URp[2] = {last ? a.eye : stkU(c, 0, jr), last ? a.eye : stkU(c, 1, jr)};
          const double* dRp[2] = {last ? a.ones : stkD(c, 0, jr), last ? a.ones : stkD(c, 1, jr)};
          const double* TRp[2] = {last ? a.eye : stkT(c, 0, jr), last ? a.eye : stkT(c, 1, jr)};
          const double* ULc[2] = {Ud[0], Ud[1]};
          const double* dLc[2] = {Dd[0], Dd[1]};
          const double* TLc[2] = {Td[0], Td[1]};
          double drift, ld[2];
          fresh_both(c, L, ULc, dLc, TLc, URp, dRp, TRp, last, &drift, ld);
          if (tid == 0) {
            ChainStats* st = c.st;
            if (drift > st->max_drift || drift != drift) st->max_drift = drift;
            if (!(drift <= a.drift_limit)) st->flags |= FLAG_DRIFT;
            for (int sp = 0; sp < 2; ++sp) {
              double e = fabs(ld[sp] - ldrun[sp]);
              if (e > st->max_logdet_err) st->max_logdet_err = e;
              ldrun[sp] = ld[sp];
            }
          }
          __syncthreads();
          clk.stop(c.st, PH_FRESH);
          cur ^= 1;
          l_prev = l;
        }
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
};

}  // namespace fast
}  // namespace dqmc
