// Implementation of the CPU emulation layer declared in hipemu.h (tests only).
// The threads of a block run as user-space fibers (ucontext) on one OS
// thread; __syncthreads switches back to a scheduler that resumes every
// fiber in turn, so a barrier completes when all fibers have reached it.
#include "hipemu.h"

#include <ucontext.h>

#include <cstring>
#include <mutex>
#include <unordered_map>

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

namespace hipemu {

thread_local dim3 tl_threadIdx, tl_blockIdx;
dim3 g_blockDim, g_gridDim;
long long g_fail_alloc_after = -1;

namespace {
constexpr size_t kStack = 256 * 1024;
enum State { RUN = 0, AT_BLOCK = 1, AT_WAVE = 2, DONE = 3 };
struct Fiber {
  ucontext_t ctx;
  char* stack = nullptr;
  int state = RUN;
};
ucontext_t sched_ctx;
std::vector<Fiber> fibers;
unsigned cur = 0;
unsigned nthreads = 1;
const std::function<void()>* g_body = nullptr;
std::vector<double> shfl_buf;
std::vector<double> mfma_buf;
std::vector<unsigned char> dyn;
#if EMU_ASAN
void* sched_fake = nullptr;
const void* sched_bottom = nullptr;
size_t sched_size = 0;
#endif

void to_scheduler(bool finishing) {
#if EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(finishing ? nullptr : &fake, sched_bottom, sched_size);
#endif
  swapcontext(&fibers[cur].ctx, &sched_ctx);
#if EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
}

void fiber_entry() {
#if EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
#endif
  (*g_body)();
  fibers[cur].state = DONE;
  to_scheduler(true);
}

void resume(unsigned t) {
  cur = t;
  const dim3 b = g_blockDim;
  tl_threadIdx = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
#if EMU_ASAN
  __sanitizer_start_switch_fiber(&sched_fake, fibers[t].stack, kStack);
#endif
  swapcontext(&sched_ctx, &fibers[t].ctx);
#if EMU_ASAN
  __sanitizer_finish_switch_fiber(sched_fake, nullptr, nullptr);
#endif
}

void wave_barrier() {
  fibers[cur].state = AT_WAVE;
  to_scheduler(false);
}

// Run every fiber of the block to completion, releasing block barriers when
// every live thread waits at one and wave barriers when every live lane of
// that wave waits at one.
void run_block(unsigned nt) {
  for (;;) {
    bool progressed = false;
    for (unsigned t = 0; t < nt; ++t)
      if (fibers[t].state == RUN) {
        resume(t);
        progressed = true;
      }
    if (progressed) continue;
    unsigned live = 0, at_block = 0;
    for (unsigned t = 0; t < nt; ++t) {
      if (fibers[t].state != DONE) ++live;
      if (fibers[t].state == AT_BLOCK) ++at_block;
    }
    if (live == 0) return;
    bool released = false;
    for (unsigned w0 = 0; w0 < nt; w0 += 64) {
      const unsigned w1 = std::min(nt, w0 + 64);
      unsigned lv = 0, aw = 0;
      for (unsigned t = w0; t < w1; ++t) {
        if (fibers[t].state != DONE) ++lv;
        if (fibers[t].state == AT_WAVE) ++aw;
      }
      if (aw > 0 && aw == lv) {
        for (unsigned t = w0; t < w1; ++t)
          if (fibers[t].state == AT_WAVE) fibers[t].state = RUN;
        released = true;
      }
    }
    if (released) continue;
    if (at_block == live) {
      if (live != nt) {
        fprintf(stderr, "hipemu: __syncthreads reached by %u threads while %u exited\n", live, nt - live);
        abort();
      }
      for (unsigned t = 0; t < nt; ++t) fibers[t].state = RUN;
      continue;
    }
    fprintf(stderr, "hipemu: deadlock (%u live, %u at a block barrier, the rest at wave barriers)\n", live,
            at_block);
    abort();
  }
}
}  // namespace

void barrier() {
  fibers[cur].state = AT_BLOCK;
  to_scheduler(false);
}

double shfl_down(double v, int off) {
  const unsigned tid = cur;
  shfl_buf[tid] = v;
  wave_barrier();
  const unsigned lane = tid & 63u;
  const double r = (lane + (unsigned)off < 64u && tid + (unsigned)off < nthreads) ? shfl_buf[tid + off] : v;
  wave_barrier();
  return r;
}

double shfl_xor(double v, int mask) {
  const unsigned tid = cur;
  shfl_buf[tid] = v;
  wave_barrier();
  const unsigned src = (tid & ~63u) | ((tid & 63u) ^ (unsigned)mask);
  const double r = src < nthreads ? shfl_buf[src] : v;
  wave_barrier();
  return r;
}

double quad_perm(double v, int ctrl) {
  if (ctrl < 0 || (ctrl >= 0x100 && ctrl != 0x140 && ctrl != 0x141)) {
    fprintf(stderr, "hipemu: only DPP quad permutations and row (half) mirrors are emulated\n");
    abort();
  }
  const unsigned tid = cur;
  shfl_buf[tid] = v;
  wave_barrier();
  const unsigned l = tid & 3u;
  unsigned src = (tid & ~3u) | ((unsigned)(ctrl >> (2 * l)) & 3u);
  if (ctrl == 0x140) src = (tid & ~15u) | (15u - (tid & 15u));  // row_mirror
  if (ctrl == 0x141) src = (tid & ~7u) | (7u - (tid & 7u));     // row_half_mirror
  const double r = src < nthreads ? shfl_buf[src] : v;
  wave_barrier();
  return r;
}

unsigned long long ballot(int pred) {
  const unsigned tid = cur;
  shfl_buf[tid] = pred ? 1.0 : 0.0;
  wave_barrier();
  const unsigned w0 = tid & ~63u;
  unsigned long long mask = 0;
  for (unsigned l = 0; l < 64 && w0 + l < nthreads; ++l)
    if (fibers[w0 + l].state != DONE && shfl_buf[w0 + l] != 0.0) mask |= 1ull << l;
  wave_barrier();
  return mask;
}

void wave_sync() { wave_barrier(); }

int readlane(int x, int lane) {
  const unsigned tid = cur;
  shfl_buf[tid] = (double)x;  // exact for every int
  wave_barrier();
  const unsigned src = (tid & ~63u) | ((unsigned)lane & 63u);
  if (lane < 0 || lane > 63 || src >= nthreads || fibers[src].state == DONE) {
    fprintf(stderr, "hipemu: readlane of lane %d, which is not live\n", lane);
    abort();
  }
  const int r = (int)shfl_buf[src];
  wave_barrier();
  return r;
}

double wave_reduce_add(double v) {
  const unsigned tid = cur;
  shfl_buf[tid] = v;
  wave_barrier();
  const unsigned w0 = tid & ~63u;
  double s = 0.0;
  for (unsigned l = 0; l < 64 && w0 + l < nthreads; ++l)
    if (fibers[w0 + l].state != DONE) s += shfl_buf[w0 + l];
  wave_barrier();
  return s;
}

d4 mfma_f64_16x16x4(double a, double b, d4 c) {
  const unsigned tid = cur;
  if (mfma_buf.size() < 2 * (size_t)nthreads) mfma_buf.assign(2 * (size_t)nthreads, 0.0);
  mfma_buf[2 * tid] = a;
  mfma_buf[2 * tid + 1] = b;
  wave_barrier();
  const unsigned w0 = tid & ~63u, l = tid & 63u;
  if (w0 + 64 > nthreads) {
    fprintf(stderr, "hipemu: MFMA in a partial wave\n");
    abort();
  }
  d4 d = c;
  for (int i = 0; i < 4; ++i) {
    const unsigned m = l / 16 + 4 * i, n = l % 16;
    double s = 0.0;
    for (unsigned k = 0; k < 4; ++k) s += mfma_buf[2 * (w0 + m + 16 * k)] * mfma_buf[2 * (w0 + n + 16 * k) + 1];
    d[i] += s;
  }
  wave_barrier();
  return d;
}

void* dyn_lds() { return dyn.data(); }

// blocks launched so far, and the block in which each static LDS variable
// was last filled
unsigned long long g_block_seq = 0;
std::unordered_map<void*, unsigned long long> g_lds_block;

void lds_fresh(void* p, size_t n) {
  unsigned long long& b = g_lds_block[p];
  if (b == g_block_seq) return;
  b = g_block_seq;
  memset(p, 0xff, n);
}

void launch(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body) {
  static std::mutex mu;  // one launch at a time (the fibers and LDS are shared)
  std::lock_guard<std::mutex> hold(mu);
  g_gridDim = grid;
  g_blockDim = block;
  const unsigned nt = block.x * block.y * block.z;
  nthreads = nt;
  g_body = &body;
  shfl_buf.assign(nt, 0.0);
  if (fibers.size() < nt) fibers.resize(nt);
  for (unsigned t = 0; t < nt; ++t)
    if (!fibers[t].stack) fibers[t].stack = (char*)malloc(kStack);
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        tl_blockIdx = dim3(bx, by, bz);
        dyn.assign(shmem ? shmem : 8, 0xff);  // LDS is not zeroed on the device
        ++g_block_seq;
        for (unsigned t = 0; t < nt; ++t) {
          getcontext(&fibers[t].ctx);
          fibers[t].ctx.uc_stack.ss_sp = fibers[t].stack;
          fibers[t].ctx.uc_stack.ss_size = kStack;
          fibers[t].ctx.uc_link = nullptr;
          fibers[t].state = RUN;
          makecontext(&fibers[t].ctx, fiber_entry, 0);
        }
        run_block(nt);
      }
}

}  // namespace hipemu

static long long g_allocs = 0;

hipError_t hipMalloc(void** p, size_t n) {
  if (hipemu::g_fail_alloc_after >= 0 && g_allocs++ >= hipemu::g_fail_alloc_after) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  *p = malloc(n ? n : 1);
  if (*p) memset(*p, 0xff, n);  // device memory is not zeroed
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                            size_t height, hipMemcpyKind, hipStream_t) {
  for (size_t r = 0; r < height; ++r) memmove((char*)dst + r * dpitch, (const char*)src + r * spitch, width);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  memset(dst, v, n);
  return hipSuccess;
}
// streams are a name only: every emulated launch runs to completion at once
hipError_t hipStreamCreate(hipStream_t* s) {
  static char token;
  *s = &token;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { return hipStreamCreate(s); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }

#include <chrono>
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new double(0.0);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
// every emulated launch has completed when its call returns
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete (double*)e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  *(double*)e = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(*(double*)b - *(double*)a);
  return hipSuccess;
}

extern "C" void hipemu_fail_alloc_after(long long k) {
  hipemu::g_fail_alloc_after = k;
  g_allocs = 0;
}

extern "C" double __ockl_wfred_add_f64(double v) { return hipemu::wave_reduce_add(v); }
