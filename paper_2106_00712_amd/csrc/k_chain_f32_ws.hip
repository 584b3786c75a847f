// chain_kernel<float, false>: the workspace-resident Green's function variant in FP32-wrap precision.
#include "k_chain.hpp"

const void* dqmc::chain_kernel_f32_ws() { return (const void*)chain_kernel<float, false>; }
