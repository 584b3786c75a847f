// fast_sweep_kernel: sweeps of chains with N <= 64 on the register/LDS path (dqmc_fast.hpp).
// Instantiated in k_fast_*.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "dqmc_fast.hpp"
#include "dqmc_kernels.hpp"

namespace dqmc {

template <int NP, typename WT, int KB>
__global__ __launch_bounds__(NT) void fast_sweep_kernel(KArgs a) {
  extern __shared__ double lds[];
  const int chain = blockIdx.x;
  if (chain >= a.n_chains) return;
  const int n_sweeps = a.counts ? a.counts[chain] : a.n_sweeps;
  if (n_sweeps <= 0) return;
  fast::Fast<NP, WT, KB>::run(a, chain, n_sweeps, lds);
}

template <int NP, typename WT, int KB>
KernelRef fast_ref() {
  return {(const void*)fast_sweep_kernel<NP, WT, KB>, fast::Fast<NP, WT, KB>::lds_bytes()};
}

}  // namespace dqmc
