// Runtime of the CPU stand-in for HIP (include/hip/hip_runtime.h): each
// workgroup runs on one OS thread and its GPU threads are fibers, switched
// by a small x86-64 context switch annotated for AddressSanitizer, at every
// workgroup barrier and wavefront exchange.  Workgroups of a grid run in
// parallel over EMU_THREADS OS threads (default 8); with EMU_REVERSE set they
// are taken in reverse order (a persistent kernel's last workgroup then
// takes the jobs, and its slot is the last one in the workspace).  The
// device reports EMU_CUS compute units (default 4).  Test infrastructure.
#include <hip/hip_runtime.h>

#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>

#include <mutex>
#include <thread>
#include <vector>

thread_local EmuIdx threadIdx;
thread_local EmuIdx blockIdx;
EmuIdx blockDim, gridDim;
thread_local char* emu_dyn_lds = nullptr;

extern "C" void emu_ctx_switch(void** save_sp, void* new_sp);
extern "C" void emu_fiber_trampoline();
asm(R"(
.text
.globl emu_ctx_switch
.type emu_ctx_switch,@function
emu_ctx_switch:
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
.size emu_ctx_switch, .-emu_ctx_switch
.globl emu_fiber_trampoline
.type emu_fiber_trampoline,@function
emu_fiber_trampoline:
  movq %r12, %rdi
  call emu_fiber_main
  ud2
.size emu_fiber_trampoline, .-emu_fiber_trampoline
)");

namespace emu {
namespace {
constexpr size_t kStack = 512 * 1024;
enum State { RUN, WAIT_BLOCK, WAIT_WAVE, DONE };
struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  State st = RUN;
  unsigned id = 0;
  EmuIdx idx{};
};
struct Sched {
  std::vector<Fiber> f;
  void* main_sp = nullptr;
  const std::function<void()>* fn = nullptr;
  unsigned n = 0;
  Fiber* cur = nullptr;
  uint64_t xbuf[16][64];
  const void* main_bottom = nullptr;
  size_t main_size = 0;
};
thread_local Sched* S = nullptr;

// switch from the running fiber back to the scheduler
void yield_to_main(State st) {
  Fiber* me = S->cur;
  me->st = st;
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, S->main_bottom, S->main_size);
  emu_ctx_switch(&me->sp, S->main_sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}
}  // namespace
}  // namespace emu

extern "C" void emu_fiber_main(emu::Fiber* f) {
  using namespace emu;
  __sanitizer_finish_switch_fiber(nullptr, &S->main_bottom, &S->main_size);
  (*S->fn)();
  f->st = DONE;
  // final switch: this fiber's fake stack may be destroyed (null save slot)
  __sanitizer_start_switch_fiber(nullptr, S->main_bottom, S->main_size);
  void* dummy;
  emu_ctx_switch(&dummy, S->main_sp);
  __builtin_unreachable();
}

namespace emu {
int lane() { return (int)(S->cur->id % 64); }

void syncthreads() {
  if (!S) { fprintf(stderr, "emu: __syncthreads outside a kernel\n"); abort(); }
  yield_to_main(WAIT_BLOCK);
}

void wave_sync() { yield_to_main(WAIT_WAVE); }

uint64_t wave_exchange(uint64_t v, int src) {
  const unsigned w = S->cur->id / 64, l = S->cur->id % 64;
  S->xbuf[w][l] = v;
  yield_to_main(WAIT_WAVE);
  if (src < 0 || src > 63) { fprintf(stderr, "emu: lane %d out of range\n", src); abort(); }
  const uint64_t r = S->xbuf[w][src];
  yield_to_main(WAIT_WAVE);
  return r;
}

int wave_all(int p) {
  const unsigned w = S->cur->id / 64, l = S->cur->id % 64;
  S->xbuf[w][l] = p ? 1 : 0;
  yield_to_main(WAIT_WAVE);
  int all = 1;
  const unsigned n = std::min(64u, S->n - w * 64);
  for (unsigned q = 0; q < n; ++q) {
    const Fiber& g = S->f[w * 64 + q];
    if (g.st != DONE && !S->xbuf[w][q]) all = 0;
  }
  yield_to_main(WAIT_WAVE);
  return all;
}

namespace {
void start_fiber(Fiber& f) {
  // initial frame: 6 callee-saved registers (r12 = the fiber) and the
  // trampoline as return address; after its ret the stack pointer is the
  // 16-byte aligned top, so the trampoline's call meets the ABI alignment
  uintptr_t top = reinterpret_cast<uintptr_t>(f.stack + kStack);
  top &= ~(uintptr_t)15;
  uint64_t* sp = reinterpret_cast<uint64_t*>(top);
  *--sp = reinterpret_cast<uint64_t>(&emu_fiber_trampoline);      // ret
  *--sp = 0;                                                      // rbp
  *--sp = 0;                                                      // rbx
  *--sp = reinterpret_cast<uint64_t>(&f);                         // r12
  *--sp = 0;                                                      // r13
  *--sp = 0;                                                      // r14
  *--sp = 0;                                                      // r15
  f.sp = sp;
}

void resume(Fiber& f) {
  S->cur = &f;
  threadIdx = f.idx;
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
  emu_ctx_switch(&S->main_sp, f.sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}

struct StackPool {
  std::vector<char*> stacks;
  char* get(unsigned i) {
    while (stacks.size() <= i) {
      void* p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
      if (p == MAP_FAILED) abort();
      stacks.push_back(static_cast<char*>(p));
    }
    return stacks[i];
  }
};
thread_local StackPool t_stacks;

void run_block(const std::function<void()>& fn, dim3 b, EmuIdx bidx, size_t shmem) {
  Sched sched;
  S = &sched;
  sched.fn = &fn;
  sched.n = b.x * b.y * b.z;
  sched.f.resize(sched.n);
  char* lds = shmem ? static_cast<char*>(malloc(shmem)) : nullptr;
  if (lds) memset(lds, 0xff, shmem);   // LDS holds garbage at a workgroup's start
  emu_dyn_lds = lds;
  blockIdx = bidx;
  for (unsigned i = 0; i < sched.n; ++i) {
    Fiber& f = sched.f[i];
    f.id = i;
    f.idx = EmuIdx{i % b.x, (i / b.x) % b.y, i / (b.x * b.y)};
    f.stack = t_stacks.get(i);
    start_fiber(f);
  }
  const unsigned nw = (sched.n + 63) / 64;
  for (;;) {
    bool ran = false;
    for (auto& f : sched.f)
      if (f.st == RUN) {
        resume(f);
        ran = true;
      }
    // release waves whose live lanes all wait at a wave barrier
    bool any_live = false, released = false;
    for (unsigned w = 0; w < nw; ++w) {
      const unsigned lo = w * 64, hi = std::min(sched.n, lo + 64);
      bool all_wave = true, live = false;
      for (unsigned q = lo; q < hi; ++q) {
        if (sched.f[q].st == DONE) continue;
        live = true;
        if (sched.f[q].st != WAIT_WAVE) all_wave = false;
      }
      if (live && all_wave) {
        for (unsigned q = lo; q < hi; ++q)
          if (sched.f[q].st == WAIT_WAVE) sched.f[q].st = RUN;
        released = true;
      }
      any_live = any_live || live;
    }
    if (!any_live) break;
    if (released) continue;
    // release the block barrier when every live thread waits at it
    bool all_block = true;
    for (auto& f : sched.f)
      if (f.st != DONE && f.st != WAIT_BLOCK) all_block = false;
    if (all_block) {
      for (auto& f : sched.f)
        if (f.st == WAIT_BLOCK) f.st = RUN;
      continue;
    }
    if (!ran) {
      fprintf(stderr, "emu: workgroup (%u,%u,%u): threads wait at different barriers\n", bidx.x,
              bidx.y, bidx.z);
      abort();
    }
  }
  free(lds);
  emu_dyn_lds = nullptr;
  S = nullptr;
}

std::mutex g_launch_mu;
}  // namespace


void run_grid(dim3 g, dim3 b, size_t shmem, const std::function<void()>& fn) {
  std::lock_guard<std::mutex> lock(g_launch_mu);
  const unsigned nt = b.x * b.y * b.z;
  if (nt == 0 || nt > 1024) { fprintf(stderr, "emu: block of %u threads\n", nt); abort(); }
  if (g.x == 0 || g.y == 0 || g.z == 0) return;
  blockDim = EmuIdx{b.x, b.y, b.z};
  gridDim = EmuIdx{g.x, g.y, g.z};
  const long total = (long)g.x * g.y * g.z;
  const char* env = getenv("EMU_THREADS");
  const int nthr = (int)std::max<long>(1, std::min<long>(env ? atoi(env) : 8, total));
  const bool rev = getenv("EMU_REVERSE") != nullptr;
  std::atomic<long> next{0};
  auto work = [&]() {
    for (;;) {
      const long k = next.fetch_add(1);
      if (k >= total) break;
      const long kk = rev ? total - 1 - k : k;
      const unsigned x = kk % g.x, y = (kk / g.x) % g.y, z = kk / ((long)g.x * g.y);
      run_block(fn, b, EmuIdx{x, y, z}, shmem);
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nthr; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}
}  // namespace emu

// ---- host API
hipError_t hipMalloc(void** p, size_t n) {
  void* q = nullptr;
  if (posix_memalign(&q, 256, n ? n : 1) != 0) return hipErrorOutOfMemory;
  memset(q, 0xcd, n);
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipPeekAtLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = malloc(1);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  free(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  const char* s = getenv("EMU_CUS");
  *v = s ? atoi(s) : 4;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
