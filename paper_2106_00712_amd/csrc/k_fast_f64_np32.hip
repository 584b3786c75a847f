// fast_sweep_kernel at NP = 32 (FP64): blocks of 8 or 16 sites.
#include "k_fast.hpp"

dqmc::KernelRef dqmc::fast_kernel_f64_np32(int kb) {
  return kb == 8 ? fast_ref<32, double, 8>() : fast_ref<32, double, 16>();
}
