// Fiber runtime of the test-only host emulation (emu_hip.h): every work-item of a workgroup is a
// fiber on one OS thread, switched by a minimal x86-64 context switch at barriers and wavefront
// collectives.  With EMU_TSAN the fibers are ThreadSanitizer fibers (a switch into a fiber carries
// the scheduler's history, a switch out carries nothing) and each barrier generation is a
// release/acquire pair; with EMU_ASAN the stack switches are announced to AddressSanitizer.
#include <sys/mman.h>

#include "emu_hip.h"

#if defined(EMU_TSAN)
extern "C" {
void* __tsan_get_current_fiber(void);
void* __tsan_create_fiber(unsigned flags);
void __tsan_destroy_fiber(void* fiber);
void __tsan_switch_to_fiber(void* fiber, unsigned flags);
void __tsan_acquire(void* addr);
void __tsan_release(void* addr);
}
#endif
#if defined(EMU_ASAN)
extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old);
}
#endif

// void emu_switch(void** save_sp, void* new_sp): saves the callee-saved registers on the current
// stack, stores its pointer, loads the other stack and restores its registers.
asm(R"(
.text
.globl emu_switch
.type emu_switch,@function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_switch,.-emu_switch
)");
extern "C" void emu_switch(void** save_sp, void* new_sp);

namespace emu {

U3 t_idx, b_idx;
Block* t_block = nullptr;
U3 g_dim, blk_dim;

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  size_t stack_size = 0;
  U3 tid;
  int state = 0;          // 0 runnable, 1 waiting, 2 done
  Barrier* wait_on = nullptr;
  long wait_gen = 0;
  void* tsan = nullptr;
  void* fake = nullptr;
};

Fiber* cur_fiber = nullptr;
static void* sched_sp = nullptr;
static const std::function<void()>* g_body = nullptr;
static const void* main_bottom = nullptr;
static size_t main_size = 0;
static void* main_tsan = nullptr;
static void* main_fake = nullptr;

void tsan_release(void* a) {
#if defined(EMU_TSAN)
  __tsan_release(a);
#else
  (void)a;
#endif
}
void tsan_acquire(void* a) {
#if defined(EMU_TSAN)
  __tsan_acquire(a);
#else
  (void)a;
#endif
}

__attribute__((no_sanitize("thread"))) static void to_scheduler(Fiber* f, bool dying) {
#if defined(EMU_TSAN)
  __tsan_switch_to_fiber(main_tsan, 1);
#endif
#if defined(EMU_ASAN)
  __sanitizer_start_switch_fiber(dying ? nullptr : &f->fake, main_bottom, main_size);
#else
  (void)dying;
#endif
  emu_switch(&f->sp, sched_sp);
#if defined(EMU_ASAN)
  __sanitizer_finish_switch_fiber(f->fake, nullptr, nullptr);
#endif
}

__attribute__((no_sanitize("thread"))) void fiber_wait(Barrier* b) {
  Fiber* f = cur_fiber;
  f->state = 1;
  f->wait_on = b;
  f->wait_gen = b->gen_;
  to_scheduler(f, false);
}

static char blk_done;
extern "C" __attribute__((no_sanitize("thread"))) void emu_trampoline() {
#if defined(EMU_ASAN)
  __sanitizer_finish_switch_fiber(nullptr, &main_bottom, &main_size);
#endif
  (*g_body)();
  Fiber* f = cur_fiber;
  f->state = 2;
  t_block->waves[f->tid.x >> 6]->bar.retire();
  t_block->bar.retire();
  tsan_release(&blk_done);
  to_scheduler(f, true);
  std::abort();   // never resumed
}

__attribute__((no_sanitize("thread"))) static void run_block(Block& blk, unsigned b, const std::function<void()>& body) {
  const int nt = blk.nthreads;
  const size_t ss = 8u << 20;   // sanitizer builds inline the kernels into frames of several hundred KB
  std::vector<Fiber> fs(nt);
  for (int t = 0; t < nt; ++t) {
    Fiber& f = fs[t];
    f.stack_size = ss;
    f.stack = (char*)mmap(nullptr, ss, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (f.stack == MAP_FAILED) { std::perror("mmap"); std::abort(); }
    f.tid.x = (unsigned)t;
    uintptr_t top = ((uintptr_t)f.stack + ss) & ~(uintptr_t)15;
    void** sp = (void**)top;
    *--sp = nullptr;                          // keeps rsp = 8 (mod 16) at the trampoline's entry
    *--sp = (void*)&emu_trampoline;           // return address of the first switch
    for (int r = 0; r < 6; ++r) *--sp = nullptr;
    f.sp = sp;
#if defined(EMU_TSAN)
    f.tsan = __tsan_create_fiber(0);
#endif
  }
  g_body = &body;
  t_block = &blk;
  b_idx.x = b;
  int left = nt, pos = 0;
  while (left > 0) {
    int scanned = 0;
    Fiber* f = nullptr;
    while (scanned < nt) {
      Fiber& c = fs[pos];
      pos = (pos + 1) % nt;
      ++scanned;
      if (c.state == 2) continue;
      if (c.state == 1) {
        if (c.wait_on->gen_ == c.wait_gen) continue;
        c.state = 0;
      }
      f = &c;
      break;
    }
    if (!f) {
      std::fprintf(stderr, "emu: deadlock in block %u:", b);
      for (int t = 0; t < nt; ++t)
        if (fs[t].state == 1) std::fprintf(stderr, " %d", t);
      std::fprintf(stderr, "\n");
      std::abort();
    }
    cur_fiber = f;
    t_idx = f->tid;
#if defined(EMU_TSAN)
    __tsan_switch_to_fiber(f->tsan, 0);
#endif
#if defined(EMU_ASAN)
    __sanitizer_start_switch_fiber(&main_fake, f->stack, f->stack_size);
#endif
    emu_switch(&sched_sp, f->sp);
#if defined(EMU_ASAN)
    __sanitizer_finish_switch_fiber(main_fake, nullptr, nullptr);
#endif
    if (f->state == 2) --left;
  }
  tsan_acquire(&blk_done);
  for (auto& f : fs) {
#if defined(EMU_TSAN)
    __tsan_destroy_fiber(f.tsan);
#endif
    munmap(f.stack, f.stack_size);
  }
}

void run_grid(Dim3 grid, Dim3 block, size_t lds, const std::function<void()>& body) {
#if defined(EMU_TSAN)
  if (!main_tsan) main_tsan = __tsan_get_current_fiber();
#endif
  const int nt = (int)(block.x * block.y * block.z);
  g_dim.x = grid.x; g_dim.y = grid.y; g_dim.z = grid.z;
  blk_dim.x = block.x; blk_dim.y = block.y; blk_dim.z = block.z;
  for (unsigned b = 0; b < grid.x; ++b) {
    Block blk;
    blk.nthreads = nt;
    blk.bar.init(nt);
    for (int w = 0; w < (nt + 63) / 64; ++w) {
      blk.waves.emplace_back(new Wave);
      const int sz = std::min(64, nt - 64 * w);
      blk.waves.back()->size = sz;
      blk.waves.back()->bar.init(sz);
    }
    blk.dyn_bytes = lds;
    if (lds) {
      blk.dyn.reset(new char[lds]);
      static const char* fe = std::getenv("EMU_LDS_FILL");
      const int fill = fe ? (int)std::strtol(fe, nullptr, 0) : 0x7f;
      if (fill >= 0) {
        std::memset(blk.dyn.get(), fill, lds);   // stands for uninitialised LDS
      } else {                                   // pseudo-random bytes
        uint64_t x = 0x9E3779B97F4A7C15ull + b;
        for (size_t i = 0; i < lds; ++i) { x ^= x << 13; x ^= x >> 7; x ^= x << 17; blk.dyn[i] = (char)x; }
      }
    }
    run_block(blk, b, body);
  }
}

}  // namespace emu
