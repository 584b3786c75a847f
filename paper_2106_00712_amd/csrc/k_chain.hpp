// chain_kernel: one workgroup per chain for every operation of a batch (init, sweeps of the
// workspace path, fixed-field probes).  Instantiated in k_chain_*.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "dqmc_device.hpp"
#include "dqmc_kernels.hpp"

namespace dqmc {

template <typename WT, bool SMALL>
__global__ __launch_bounds__(NT) void chain_kernel(KArgs a) {
  extern __shared__ double lds[];
  const int idx = blockIdx.x;
  const int chain = a.slots ? a.slots[idx] : idx;
  if (chain < 0 || chain >= a.n_chains) return;
  const int n_sweeps = a.counts ? a.counts[chain] : a.n_sweeps;
  if (a.op == OP_SWEEP && n_sweeps <= 0) return;
  Ctx<WT> c = make_ctx<WT, SMALL>(a, chain, lds);
  if (a.op == OP_INIT) {
    if (threadIdx.x == 0) {
      ChainStats* st = c.st;
      st->seed = a.seeds[idx];
      st->sweeps_done = st->attempted = st->accepted = st->near_ties = 0;
      st->max_drift = st->max_logdet_err = 0.0;
      st->logdet[0] = st->logdet[1] = 0.0;
      st->flags = 0;
      st->pad = 0;
      for (int k = 0; k < 16; ++k) st->ticks[k] = 0;
      st->slice_docc = st->slice_kin = 0.0;
      st->slice_meas = 0;
      st->stack_ok = 0;
      st->pad2 = 0;
    }
    __syncthreads();
    op_init(c, idx);
  } else if (a.op == OP_SWEEP) {
    op_sweep(c, n_sweeps);
  } else if (a.op == OP_DEBUG_GREEN) {
    op_debug_green(c, chain);
  } else if (a.op == OP_DEBUG_RATIOS) {
    op_debug_ratios(c, chain);
  }
}

}  // namespace dqmc
