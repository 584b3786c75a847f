// Streams of the caller's own for batches that run side by side (dqmc_stream_create/destroy).
#include <hip/hip_runtime.h>

#include <string>

#include "dqmc.h"
#include "dqmc_error.hpp"

dqmc_status dqmc_stream_create(void** out) {
  if (!out) return dqmc::set_error(DQMC_EINVAL, "out is NULL");
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess)
    return dqmc::set_error(DQMC_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
  *out = (void*)s;
  return DQMC_OK;
}

dqmc_status dqmc_stream_destroy(void* stream) {
  if (!stream) return dqmc::set_error(DQMC_EINVAL, "stream is NULL");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamDestroy((hipStream_t)stream);
  if (e != hipSuccess)
    return dqmc::set_error(DQMC_EDEVICE, std::string("dqmc_stream_destroy: ") + hipGetErrorString(e));
  return DQMC_OK;
}
