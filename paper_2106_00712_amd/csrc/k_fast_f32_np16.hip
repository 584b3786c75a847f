// fast_sweep_kernel at NP = 16 (FP32-wrap): one block size, 8 sites.
#include "k_fast.hpp"

dqmc::KernelRef dqmc::fast_kernel_f32_np16(int) { return fast_ref<16, float, 8>(); }
