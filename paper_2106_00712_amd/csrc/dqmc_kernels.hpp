// The sweep kernels of the library live in translation units of their own (one per group of
// template instantiations, so that they compile in parallel); the host side (dqmc_abi.hip)
// reaches them through the accessors declared here.
#pragma once
#include <cstddef>

namespace dqmc {

struct KernelRef {
  const void* fn;   // host stub of the __global__ function (argument of hipLaunchKernel)
  size_t lds;       // dynamic LDS bytes the kernel needs (0: given by the caller)
};

// chain_kernel<WT, SMALL>: init, sweeps and probes at any N (k_chain_*.hip)
const void* chain_kernel_f64_lds();
const void* chain_kernel_f64_ws();
const void* chain_kernel_f32_lds();
const void* chain_kernel_f32_ws();

// fast_sweep_kernel<NP, WT, KB>: sweeps at NP in {16, 32, 64} (k_fast_*.hip)
KernelRef fast_kernel_f64_np16(int kb);
KernelRef fast_kernel_f64_np32(int kb);
KernelRef fast_kernel_f64_np64(int kb);
KernelRef fast_kernel_f32_np16(int kb);
KernelRef fast_kernel_f32_np32(int kb);
KernelRef fast_kernel_f32_np64(int kb);

}  // namespace dqmc
