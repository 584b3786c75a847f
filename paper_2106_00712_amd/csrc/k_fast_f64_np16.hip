// fast_sweep_kernel at NP = 16 (FP64): one block size, 8 sites.
#include "k_fast.hpp"

dqmc::KernelRef dqmc::fast_kernel_f64_np16(int) { return fast_ref<16, double, 8>(); }
