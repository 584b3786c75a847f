// Test-only host emulation of the HIP subset the library's kernels use, so that the kernel
// sources can run on the CPU under AddressSanitizer and ThreadSanitizer and be compared with the
// oracle without a GPU.  It is never built into the package (which loads libdqmc.so built for
// gfx950 and fails without it).
//
// Model: every work-item of a workgroup is a fiber on one OS thread (emu_rt.cpp).  Workgroup
// barriers and the wavefront collectives (readlane, shuffles, ballot, DPP row operations, the
// 16x16x4 MFMA products) are barriers of the fibers, and the wavefront-ordering points of the
// kernels (s_waitcnt on LDS, the compiler barrier that orders a wavefront's LDS accesses) become
// wavefront barriers.  Everything else a work-item does runs unsynchronised, so ThreadSanitizer
// reports any pair of accesses from different work-items that no barrier orders.  Workgroups run
// one after another.
#pragma once
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace emu {

struct U3 {
  unsigned x = 0, y = 0, z = 0;
};
struct Dim3 {
  unsigned x, y, z;
  Dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct Fiber;
struct Barrier;
extern Fiber* cur_fiber;
void fiber_wait(Barrier* b);     // suspend the current fiber until b releases
void tsan_release(void* a);
void tsan_acquire(void* a);

// Workgroup or wavefront barrier among fibers (one OS thread runs every work-item of a block).
struct Barrier {
  int n_ = 0, count_ = 0;
  long gen_ = 0;
  char sync_[2];    // per-generation addresses for the sanitizer's happens-before edges
  void init(int n) { n_ = n; }
  __attribute__((no_sanitize("thread"))) void retire() {
    --n_;
    if (count_ > 0 && count_ >= n_) { count_ = 0; ++gen_; }
  }
  __attribute__((no_sanitize("thread"))) void wait(const char*) {
    const long g = gen_;
    tsan_release(&sync_[g & 1]);
    if (++count_ >= n_) {
      count_ = 0;
      ++gen_;
    } else {
      fiber_wait(this);
    }
    tsan_acquire(&sync_[g & 1]);
  }
};

// Exchange buffers of the wavefront collectives, double-buffered: collective k uses buffer k % 2,
// so one barrier per collective suffices (a lane can only reach collective k + 2, which writes
// buffer k % 2 again, after every lane has passed collective k + 1, i.e. finished reading k).
struct Wave {
  Barrier bar;
  int size = 64;
  int seq[64] = {};
  uint64_t slot[2][64];
  double a64[2][64], b64[2][64];
  float a32[2][64], b32[2][64];
};

struct Block {
  Barrier bar;
  std::vector<std::unique_ptr<Wave>> waves;
  std::unique_ptr<char[]> dyn;
  size_t dyn_bytes = 0;
  int nthreads = 0;
};

extern U3 t_idx;
extern U3 b_idx;
extern Block* t_block;
extern U3 g_dim, blk_dim;

inline int lane_id() { return (int)(t_idx.x & 63); }
inline Wave& my_wave() { return *t_block->waves[t_idx.x >> 6]; }

inline void sync_block() { t_block->bar.wait("__syncthreads"); }
inline void wave_sync() { my_wave().bar.wait("wave sync"); }

template <typename T>
inline uint64_t to_bits(T v) {
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <typename T>
inline T from_bits(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}

// all lanes publish a value; returns a copy of the wave's 64 values
inline int next_buffer(Wave& w) { return w.seq[lane_id()]++ & 1; }

template <typename T>
inline void gather(T v, uint64_t out[64]) {
  Wave& w = my_wave();
  const int q = next_buffer(w);
  w.slot[q][lane_id()] = to_bits(v);
  w.bar.wait("gather");
  std::memcpy(out, w.slot[q], sizeof(uint64_t) * 64);
}

template <typename T>
inline T readlane(T v, int src) {
  uint64_t all[64];
  gather(v, all);
  return from_bits<T>(all[src & 63]);
}
template <typename T>
inline T shfl(T v, int src) { return readlane(v, src); }
template <typename T>
inline T shfl_xor(T v, int mask) { return readlane(v, lane_id() ^ mask); }

inline unsigned long long ballot(int pred) {
  uint64_t all[64];
  gather<int>(pred ? 1 : 0, all);
  unsigned long long m = 0;
  const int n = my_wave().size;
  for (int l = 0; l < n; ++l)
    if (from_bits<int>(all[l])) m |= 1ull << l;
  return m;
}

inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  uint64_t all[64];
  gather(src, all);
  const int l = lane_id(), r = l >> 4, i = l & 15;
  if (!((row_mask >> r) & 1) || !((bank_mask >> (i >> 2)) & 1)) return old;
  int s = -1;
  if (ctrl >= 0x111 && ctrl <= 0x11F) {            // row_shr:k
    const int k = ctrl - 0x110;
    if (i >= k) s = l - k;
  } else if (ctrl >= 0x101 && ctrl <= 0x10F) {     // row_shl:k
    const int k = ctrl - 0x100;
    if (i + k < 16) s = l + k;
  } else if (ctrl >= 0x121 && ctrl <= 0x12F) {     // row_ror:k
    const int k = ctrl - 0x120;
    s = (l & ~15) | ((i + k) & 15);
  } else if (ctrl == 0x142) {                      // row_bcast:15
    if (r >= 1) s = 16 * r - 1;
  } else if (ctrl == 0x143) {                      // row_bcast:31
    if (r >= 2) s = 31;
  } else if (ctrl < 0x100) {                       // quad_perm
    s = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
  } else {
    std::fprintf(stderr, "emu: DPP control 0x%x not emulated\n", ctrl);
    std::abort();
  }
  if (s < 0) return bound_ctrl ? 0 : old;
  return from_bits<int>(all[s]);
}

// MFMA instructions issued (one per wavefront), FP64 and FP32: work counters of the emulation.
inline long long& mfma_issued(int fp32) {
  static long long n[2] = {0, 0};
  return n[fp32];
}

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// acc += A(16x4) B(4x16); lane l supplies A[l%16][l/16] and B[l/16][l%16]; FP64 output register v
// of lane l holds row 4v + l/16, FP32 output register v holds row 4(l/16) + v, column l%16.
inline d4v mfma_f64(double a, double b, d4v c) {
  Wave& w = my_wave();
  const int l = lane_id(), q = next_buffer(w);
  if (l == 0) __atomic_fetch_add(&mfma_issued(0), 1, __ATOMIC_RELAXED);
  w.a64[q][l] = a;
  w.b64[q][l] = b;
  w.bar.wait("mfma");
  d4v out;
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * v + (l >> 4), col = l & 15;
    double s = c[v];
    for (int k = 0; k < 4; ++k) s = std::fma(w.a64[q][16 * k + row], w.b64[q][16 * k + col], s);
    out[v] = s;
  }
  return out;
}
inline f4v mfma_f32(float a, float b, f4v c) {
  Wave& w = my_wave();
  const int l = lane_id(), q = next_buffer(w);
  if (l == 0) __atomic_fetch_add(&mfma_issued(1), 1, __ATOMIC_RELAXED);
  w.a32[q][l] = a;
  w.b32[q][l] = b;
  w.bar.wait("mfma32");
  f4v out;
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * (l >> 4) + v, col = l & 15;
    float s = c[v];
    for (int k = 0; k < 4; ++k) s = std::fma(w.a32[q][16 * k + row], w.b32[q][16 * k + col], s);
    out[v] = s;
  }
  return out;
}

inline int64_t clock64() {
  static std::atomic<int64_t> c{0};
  return c.fetch_add(1, std::memory_order_relaxed);
}

inline double* dyn_lds() { return (double*)t_block->dyn.get(); }

void run_grid(Dim3 grid, Dim3 block, size_t lds, const std::function<void()>& body);

}  // namespace emu

// ------------------------------------------------------------------ device-side names
#define threadIdx emu::t_idx
#define blockIdx emu::b_idx
inline emu::U3& gridDim = emu::g_dim;
inline emu::U3& blockDim = emu::blk_dim;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__ static
#define __syncthreads() emu::sync_block()
#define __shfl(v, s) emu::shfl((v), (s))
#define __shfl_xor(v, m) emu::shfl_xor((v), (m))
#define __ballot(p) emu::ballot(p)
#define __builtin_amdgcn_readlane(v, l) emu::readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) emu::readlane((v), 0)
#define __builtin_amdgcn_update_dpp(o, s, c, r, b, bc) emu::update_dpp((o), (s), (c), (r), (b), (bc))
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu::mfma_f64((a), (b), (c))
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu::mfma_f32((a), (b), (c))
#define wall_clock64() emu::clock64()

#include <type_traits>
template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) { return a < b ? a : b; }
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) { return a < b ? b : a; }
inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
inline int __double2loint(double d) { return (int)(uint32_t)emu::to_bits(d); }
inline int __double2hiint(double d) { return (int)(uint32_t)(emu::to_bits(d) >> 32); }
inline double __hiloint2double(int hi, int lo) {
  return emu::from_bits<double>(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicOr(unsigned* p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

// ------------------------------------------------------------------ host API
typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef emu::Dim3 dim3;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };
enum hipDeviceAttribute_t { hipDeviceAttributeMaxSharedMemoryPerBlock };
constexpr unsigned hipStreamNonBlocking = 1;
constexpr unsigned hipEventDisableTiming = 2;

inline const char* hipGetErrorString(hipError_t) { return "emulated error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 160 * 1024; return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h,
                                   hipMemcpyKind, hipStream_t) {
  for (size_t r = 0; r < h; ++r) std::memmove((char*)d + r * dp, (const char*)s + r * sp, w);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  std::memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new int(0); return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete (int*)s; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new int(0); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
#define HIP_SYMBOL(x) ((const void*)&(x))

// kernels launched through a pointer take one argument (the library's KArgs), by value; the
// driver defines how to call them
void emu_call_kernel(const void* fn, void** params);
inline hipError_t hipLaunchKernel(const void* fn, dim3 g, dim3 b, void** params, size_t lds, hipStream_t) {
  void* p0 = params[0];
  emu::run_grid(g, b, lds, [fn, p0] {
    void* ps[1] = {p0};
    emu_call_kernel(fn, ps);
  });
  return hipSuccess;
}
#define hipLaunchKernelGGL(k, g, b, lds, s, ...) emu::run_grid((g), (b), (lds), [=] { k(__VA_ARGS__); })

// graphs: kernel nodes replayed in order
struct hipKernelNodeParams {
  void* func;
  dim3 gridDim, blockDim;
  unsigned sharedMemBytes;
  void** kernelParams;
  void** extra;
};
struct EmuNode {
  const void* fn;
  dim3 g, b;
  size_t lds;
  void* p0;
};
typedef std::vector<EmuNode>* hipGraph_t;
typedef std::vector<EmuNode>* hipGraphExec_t;
typedef int hipGraphNode_t;
inline hipError_t hipGraphCreate(hipGraph_t* g, unsigned) { *g = new std::vector<EmuNode>; return hipSuccess; }
inline hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g, void*, size_t, const hipKernelNodeParams* p) {
  g->push_back({p->func, p->gridDim, p->blockDim, p->sharedMemBytes, p->kernelParams[0]});
  *n = (int)g->size();
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
  *e = new std::vector<EmuNode>(*g);
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  for (auto& n : *e) {
    void* ps[1] = {n.p0};
    hipLaunchKernel(n.fn, n.g, n.b, ps, n.lds, s);
  }
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
