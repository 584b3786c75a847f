// fast_sweep_kernel at NP = 64 (FP32-wrap): blocks of 8 or 16 sites.
#include "k_fast.hpp"

dqmc::KernelRef dqmc::fast_kernel_f32_np64(int kb) {
  return kb == 8 ? fast_ref<64, float, 8>() : fast_ref<64, float, 16>();
}
