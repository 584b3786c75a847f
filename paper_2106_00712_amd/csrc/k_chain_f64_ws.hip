// chain_kernel<double, false>: the workspace-resident Green's function variant in FP64 precision.
#include "k_chain.hpp"

const void* dqmc::chain_kernel_f64_ws() { return (const void*)chain_kernel<double, false>; }
