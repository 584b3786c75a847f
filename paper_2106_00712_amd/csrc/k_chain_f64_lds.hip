// chain_kernel<double, true>: the LDS-resident Green's function variant in FP64 precision.
#include "k_chain.hpp"

const void* dqmc::chain_kernel_f64_lds() { return (const void*)chain_kernel<double, true>; }
