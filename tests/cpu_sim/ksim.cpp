// CPU runtime behind tests/cpu_sim/hip/hip_runtime.h (test use only).
//
// Memory: every hipMalloc block is placed so that it ends just below an
// inaccessible guard page (and starts above another), so an access out of
// bounds faults at once.  Kernels: a launch runs its blocks on CPU threads
// (at most KSIM_RESIDENT at a time, in block order); a block's threads are
// fibers on one CPU thread, switched by a small context switch at barriers,
// cross-lane operations and s_sleep.  Streams execute each operation when it
// is enqueued, or record it while a stream captures a graph.
#include "hip/hip_runtime.h"

#include <execinfo.h>
#include <sched.h>
#include <signal.h>
#include <sys/mman.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

// ------------------------------------------------------------------ context switch (x86-64 SysV)
extern "C" void ksim_switch(void** save_sp, void* load_sp);
extern "C" void ksim_trampoline();
asm(R"(
  .text
  .globl ksim_switch
  .type ksim_switch,@function
ksim_switch:
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
  .globl ksim_trampoline
  .type ksim_trampoline,@function
ksim_trampoline:
  movq %r12, %rdi
  call ksim_fiber_main
  ud2
)");

namespace {

// A fault prints the address and the call stack (on an alternate stack, so
// that a fiber's overflowed stack can be reported too).
void on_fault(int sig, siginfo_t* si, void*) {
  char buf[128];
  const int n = snprintf(buf, sizeof buf, "ksim: signal %d at address %p\n", sig, si->si_addr);
  (void)!write(2, buf, (size_t)n);
  void* frames[64];
  const int nf = backtrace(frames, 64);
  backtrace_symbols_fd(frames, nf, 2);
  _exit(128 + sig);
}

struct FaultHandler {
  FaultHandler() {
    static char alt[1 << 16];
    stack_t ss;
    ss.ss_sp = alt;
    ss.ss_size = sizeof alt;
    ss.ss_flags = 0;
    sigaltstack(&ss, nullptr);
    struct sigaction sa;
    memset(&sa, 0, sizeof sa);
    sa.sa_sigaction = on_fault;
    sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
    sigaction(SIGSEGV, &sa, nullptr);
    sigaction(SIGBUS, &sa, nullptr);
  }
} g_fault_handler;

size_t page() {
  static const size_t p = (size_t)sysconf(_SC_PAGESIZE);
  return p;
}

[[noreturn]] void die(const char* msg) {
  fprintf(stderr, "ksim: %s\n", msg);
  fflush(stderr);
  abort();
}

long env_long(const char* name, long def) {
  const char* s = getenv(name);
  return s && *s ? strtol(s, nullptr, 10) : def;
}

// ------------------------------------------------------------------ guarded memory
struct Mapping {
  void* base;
  size_t len;
};
// never destroyed: the library frees its cached buffers from static destructors
std::mutex& g_mem_mu = *new std::mutex;
std::map<void*, Mapping>& g_mem = *new std::map<void*, Mapping>;

void* guarded_alloc(size_t bytes) {
  const size_t P = page();
  const size_t body = (std::max<size_t>(bytes, 1) + P - 1) / P * P;
  const size_t len = body + 2 * P;
  void* base = mmap(nullptr, len, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (base == MAP_FAILED) return nullptr;
  if (mprotect((char*)base + P, body, PROT_READ | PROT_WRITE) != 0) {
    munmap(base, len);
    return nullptr;
  }
  // end the block within 256 bytes of the upper guard page
  const size_t used = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  char* p = (char*)base + P + (body - used);
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_mem[p] = Mapping{base, len};
  return p;
}

bool guarded_free(void* p) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_mem.find(p);
  if (it == g_mem.end()) return false;
  munmap(it->second.base, it->second.len);
  g_mem.erase(it);
  return true;
}

// ------------------------------------------------------------------ fibers
constexpr int kWave = 64;
constexpr size_t kStack = 64 * 1024;

struct Block;

struct Fiber {
  ksim_dims dims;
  void* sp = nullptr;
  char* stack = nullptr;  // lowest usable address
  Block* blk = nullptr;
  const std::function<void()>* body = nullptr;
  bool done = false;
  int64_t coll = 0;  // collectives this lane has entered
};

struct WaveColl {
  int64_t seq[2] = {-1, -1};
  int count[2] = {0, 0};
  int kind[2] = {0, 0};
  uint64_t vals[2][kWave];
  uint64_t mask[2] = {0, 0};
};

struct Block {
  std::vector<Fiber> fibers;
  std::vector<WaveColl> waves;
  std::vector<int> wave_live;
  int live = 0;
  int arrived = 0;
  int64_t gen = 0;
  void* sched_sp = nullptr;
  int cur = -1;
};

thread_local Block* t_blk = nullptr;
thread_local ksim_dims t_host_dims;

// stacks are reused across launches: one set of up to 1024 per CPU thread
std::mutex& g_stack_mu = *new std::mutex;
std::vector<char*>& g_stack_sets = *new std::vector<char*>;

char* take_stack_set() {
  {
    std::lock_guard<std::mutex> lk(g_stack_mu);
    if (!g_stack_sets.empty()) {
      char* s = g_stack_sets.back();
      g_stack_sets.pop_back();
      return s;
    }
  }
  // 1024 stacks in one mapping (a guard page per stack would cost a memory
  // map entry each); the lowest bytes of every stack hold a canary that is
  // checked after each block
  const size_t per = kStack + page();
  char* base = (char*)mmap(nullptr, per * 1024, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1,
                           0);
  if (base == (char*)MAP_FAILED) die("no memory for fiber stacks");
  return base;
}

void give_stack_set(char* s) {
  std::lock_guard<std::mutex> lk(g_stack_mu);
  g_stack_sets.push_back(s);
}

void fiber_yield() {
  Block* b = t_blk;
  Fiber& f = b->fibers[b->cur];
  ksim_switch(&f.sp, b->sched_sp);
}

}  // namespace

extern "C" void ksim_fiber_main(Fiber* f) {
  (*f->body)();
  f->done = true;
  Block* b = f->blk;
  --b->live;
  --b->wave_live[f->dims.tid.x / kWave];
  // a barrier that now holds every remaining thread opens
  if (b->arrived > 0 && b->arrived == b->live) {
    b->arrived = 0;
    ++b->gen;
  }
  for (;;) ksim_switch(&f->sp, b->sched_sp);
}

namespace {

void run_block(const dim3& grid, const dim3& block, unsigned bx, const std::function<void()>& body, char* stacks) {
  const int nt = (int)(block.x * block.y * block.z);
  if (nt > 1024 || nt % kWave != 0) die("block size must be a multiple of 64, at most 1024");
  Block b;
  b.fibers.resize(nt);
  b.waves.resize(nt / kWave);
  b.wave_live.assign(nt / kWave, kWave);
  b.live = nt;
  const size_t per = kStack + page();
  for (int t = 0; t < nt; ++t) {
    Fiber& f = b.fibers[t];
    f.dims.tid = dim3(t, 0, 0);
    f.dims.bid = dim3(bx, 0, 0);
    f.dims.bdim = block;
    f.dims.gdim = grid;
    f.blk = &b;
    f.body = &body;
    f.stack = stacks + t * per + page();
    memcpy(f.stack - 8, "ksimcnry", 8);
    uintptr_t top = ((uintptr_t)(f.stack + kStack)) & ~(uintptr_t)15;
    uint64_t* sp = (uint64_t*)(top - 72);
    sp[0] = 0;                                  // r15
    sp[1] = 0;                                  // r14
    sp[2] = 0;                                  // r13
    sp[3] = (uint64_t)(uintptr_t)&f;            // r12: the fiber
    sp[4] = 0;                                  // rbx
    sp[5] = 0;                                  // rbp
    sp[6] = (uint64_t)(uintptr_t)&ksim_trampoline;
    f.sp = sp;
  }
  Block* saved = t_blk;
  t_blk = &b;
  int idle_rounds = 0;
  while (b.live > 0) {
    const int64_t g0 = b.gen;
    int alive = 0;
    for (int t = 0; t < nt; ++t) {
      if (b.fibers[t].done) continue;
      ++alive;
      b.cur = t;
      ksim_switch(&b.sched_sp, b.fibers[t].sp);
    }
    // every thread of this block is waiting on others (a spin in a look-back
    // or the LDS queue): let the other blocks' CPU threads run
    if (b.gen == g0 && alive > 0 && ++idle_rounds > 2) {
      sched_yield();
      idle_rounds = 0;
    }
  }
  t_blk = saved;
  for (int t = 0; t < nt; ++t)
    if (memcmp(b.fibers[t].stack - 8, "ksimcnry", 8) != 0) die("a fiber overflowed its stack");
}

// Workgroup slots of the device (KSIM_SLOTS; unset: unlimited).  A block holds
// a slot while it runs, and the blocks of a launch take slots in block order,
// so kernels on other streams that hold slots keep later blocks waiting.
struct Slots {
  std::mutex mu;
  std::condition_variable cv;
  long free = -1;  // -1: unlimited
};
Slots& g_slots = *new Slots;

void slot_take() {
  std::unique_lock<std::mutex> lk(g_slots.mu);
  if (g_slots.free < 0) return;
  g_slots.cv.wait(lk, [] { return g_slots.free > 0; });
  --g_slots.free;
}
void slot_give() {
  std::lock_guard<std::mutex> lk(g_slots.mu);
  if (g_slots.free < 0) return;
  ++g_slots.free;
  g_slots.cv.notify_all();
}

void run_grid(dim3 grid, dim3 block, const std::function<void()>& body) {
  const unsigned nb = grid.x * grid.y * grid.z;
  if (nb == 0) return;
  const long resident = env_long("KSIM_RESIDENT", 64);
  const unsigned nthreads = (unsigned)std::max<long>(1, std::min<long>(resident, nb));
  std::atomic<unsigned> next{0};
  std::mutex order_mu;  // a slot is taken, then the next block index, in order
  auto worker = [&]() {
    char* stacks = nullptr;  // taken once the worker runs a block
    for (;;) {
      unsigned bx;
      {
        std::lock_guard<std::mutex> lk(order_mu);
        if (next.load() >= nb) break;
        slot_take();
        bx = next.fetch_add(1);
      }
      if (!stacks) stacks = take_stack_set();
      run_block(grid, block, bx, body, stacks);
      slot_give();
    }
    if (stacks) give_stack_set(stacks);
  };
  std::vector<std::thread> th;
  for (unsigned k = 1; k < nthreads; ++k) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

// ------------------------------------------------------------------ streams and graphs
}  // namespace

struct ksim_graph {
  std::vector<std::function<void()>> ops;
};

namespace {

// A command of a hardware queue: work, a marker (no work) or a barrier that
// holds the queue until another command has completed.
struct Cmd {
  std::function<void()> fn;
  std::shared_ptr<Cmd> wait_for;
  std::atomic<bool> done{false};
};

// With KSIM_HWQ=Q (Q >= 1) streams map round-robin onto Q in-order queues,
// each drained by a thread of its own, as the runtime maps streams onto the
// hardware queues it has; 0 (the default) runs every command when it is
// enqueued.
struct HwQueue {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Cmd>> q;
  std::thread th;
  bool busy = false;
};

std::vector<HwQueue*>& g_hwq = *new std::vector<HwQueue*>;
std::mutex& g_hwq_mu = *new std::mutex;
std::atomic<int> g_next_q{0};

void wait_done(const std::shared_ptr<Cmd>& c) {
  while (c && !c->done.load()) std::this_thread::sleep_for(std::chrono::microseconds(20));
}

void drain(HwQueue* hq) {
  for (;;) {
    std::shared_ptr<Cmd> c;
    {
      std::unique_lock<std::mutex> lk(hq->mu);
      hq->cv.wait(lk, [&] { return !hq->q.empty(); });
      c = hq->q.front();
      hq->busy = true;
    }
    wait_done(c->wait_for);
    if (c->fn) c->fn();
    c->done.store(true);
    {
      std::lock_guard<std::mutex> lk(hq->mu);
      hq->q.pop_front();
      hq->busy = false;
    }
  }
}

int hw_queues() {
  static const int q = (int)env_long("KSIM_HWQ", 0);
  static std::once_flag once;
  std::call_once(once, [] {
    for (int k = 0; k < q; ++k) {
      HwQueue* hq = new HwQueue;
      hq->th = std::thread(drain, hq);
      hq->th.detach();
      g_hwq.push_back(hq);
    }
    const long slots = env_long("KSIM_SLOTS", -1);
    g_slots.free = slots > 0 ? slots : -1;
  });
  return q;
}

// every queue empty and idle (the device-wide synchronization of hipFree)
void device_idle() {
  if (!hw_queues()) return;
  for (;;) {
    bool idle = true;
    for (HwQueue* hq : g_hwq) {
      std::lock_guard<std::mutex> lk(hq->mu);
      idle = idle && hq->q.empty() && !hq->busy;
    }
    if (idle) return;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace

struct ksim_stream {
  ksim_graph* capture = nullptr;
  int hwq = 0;
  std::shared_ptr<Cmd> last;
};
struct ksim_event {
  std::shared_ptr<Cmd> cmd;
};

namespace {

ksim_stream& g_null_stream = *new ksim_stream;

thread_local hipError_t t_last = hipSuccess;

ksim_stream* stream_of(hipStream_t s) { return s ? s : &g_null_stream; }

std::shared_ptr<Cmd> submit(ksim_stream* st, std::function<void()> fn, std::shared_ptr<Cmd> wait_for) {
  auto c = std::make_shared<Cmd>();
  c->fn = std::move(fn);
  c->wait_for = std::move(wait_for);
  HwQueue* hq = g_hwq[(size_t)st->hwq];
  {
    std::lock_guard<std::mutex> lk(hq->mu);
    hq->q.push_back(c);
    st->last = c;
  }
  hq->cv.notify_one();
  return c;
}

void enqueue(hipStream_t s, std::function<void()> op) {
  ksim_stream* st = stream_of(s);
  if (st->capture)
    st->capture->ops.push_back(std::move(op));
  else if (!hw_queues())
    op();
  else
    submit(st, std::move(op), nullptr);
}

}  // namespace

// ------------------------------------------------------------------ device-side calls
ksim_dims* ksim_cur() {
  Block* b = t_blk;
  if (!b) return &t_host_dims;
  return &b->fibers[b->cur].dims;
}

uint32_t ksim_lane() { return ksim_cur()->tid.x % kWave; }

void ksim_yield() {
  if (t_blk) fiber_yield();
}

void __syncthreads() {
  Block* b = t_blk;
  if (!b) return;
  const int64_t my = b->gen;
  if (++b->arrived == b->live) {
    b->arrived = 0;
    ++b->gen;
    return;
  }
  while (b->gen == my) fiber_yield();
}

namespace {

enum { kBallot = 1, kReadlane, kFirst, kDpp, kSync, kShfl };

// All live lanes of the calling wave deposit v; returns the wave's values
// (and, in *mask, the lanes that deposited) once everyone has.
const uint64_t* collect(uint64_t v, int kind, uint64_t* mask) {
  Block* b = t_blk;
  Fiber& f = b->fibers[b->cur];
  const int w = f.dims.tid.x / kWave, lane = f.dims.tid.x % kWave;
  WaveColl& W = b->waves[w];
  const int64_t c = f.coll++;
  const int k = (int)(c & 1);
  if (W.seq[k] != c) {
    W.seq[k] = c;
    W.count[k] = 0;
    W.kind[k] = kind;
    W.mask[k] = 0;
  }
  if (W.kind[k] != kind) die("lanes of a wave reached different cross-lane operations");
  W.vals[k][lane] = v;
  W.mask[k] |= 1ull << lane;
  ++W.count[k];
  while (W.count[k] < b->wave_live[w]) {
    fiber_yield();
    if (W.seq[k] != c) die("cross-lane operation overtaken");
  }
  *mask = W.mask[k];
  return W.vals[k];
}

}  // namespace

void ksim_wave_sync() {
  if (!t_blk) return;
  uint64_t m;
  (void)collect(0, kSync, &m);
}

uint64_t ksim_ballot(bool pred) {
  if (!t_blk) return pred ? 1 : 0;
  uint64_t m;
  const uint64_t* v = collect(pred ? 1 : 0, kBallot, &m);
  uint64_t r = 0;
  for (int j = 0; j < kWave; ++j)
    if (((m >> j) & 1) && v[j]) r |= 1ull << j;
  return r;
}

uint64_t ksim_readlane(uint64_t x, int src) {
  if (!t_blk) return x;
  uint64_t m;
  const uint64_t* v = collect(x, kReadlane, &m);
  if (src < 0 || src >= kWave || !((m >> src) & 1)) die("readlane of an inactive lane");
  return v[src];
}

uint64_t ksim_shfl(uint64_t x, int src) {
  if (!t_blk) return x;
  uint64_t m;
  const uint64_t* v = collect(x, kShfl, &m);
  if (src < 0 || src >= kWave || !((m >> src) & 1)) die("shuffle from an inactive lane");
  return v[src];
}

uint64_t ksim_readfirstlane(uint64_t x) {
  if (!t_blk) return x;
  uint64_t m;
  const uint64_t* v = collect(x, kFirst, &m);
  return v[__builtin_ctzll(m)];
}

int ksim_dpp(int old, int x, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  if (!t_blk) return x;
  uint64_t m;
  const uint64_t* v = collect((uint64_t)(uint32_t)x, kDpp, &m);
  const int i = (int)ksim_lane(), row = i / 16, k = i % 16;
  if (!((row_mask >> row) & 1) || !((bank_mask >> (k / 4)) & 1)) return old;
  int src = -1;
  if (ctrl >= 0x111 && ctrl <= 0x11f) {  // row_shr:n
    const int n = ctrl - 0x110;
    if (k >= n) src = i - n;
  } else if (ctrl == 0x142) {  // row_bcast:15, lane 15 of each row into the next row
    if (row >= 1) src = 16 * row - 1;
  } else if (ctrl == 0x143) {  // row_bcast:31, lane 31 into rows 2 and 3
    if (row >= 2) src = 31;
  } else {
    die("unsupported DPP control");
  }
  if (src < 0 || !((m >> src) & 1)) return bound_ctrl ? 0 : old;
  return (int)(uint32_t)v[src];
}

void ksim_launch(hipStream_t s, dim3 grid, dim3 block, std::function<void()> body) {
  enqueue(s, [grid, block, body]() { run_grid(grid, block, body); });
}

// ------------------------------------------------------------------ host API
hipError_t hipMalloc(void** p, size_t bytes) {
  *p = guarded_alloc(bytes);
  return *p ? hipSuccess : (t_last = hipErrorOutOfMemory);
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  device_idle();  // the runtime synchronizes the device before a free
  return guarded_free(p) ? hipSuccess : (t_last = hipErrorInvalidValue);
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = guarded_alloc(bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (!hw_queues()) {
    memcpy(dst, src, bytes);
    return hipSuccess;
  }
  // ordered on the null stream, and the host waits for it
  wait_done(submit(&g_null_stream, [=]() { memcpy(dst, src, bytes); }, nullptr));
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  enqueue(s, [=]() { memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s) {
  enqueue(s, [=]() { memset(dst, value, bytes); });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ksim_stream;
  const int q = hw_queues();
  if (q) (*s)->hwq = (1 + g_next_q.fetch_add(1)) % q;  // the null stream has queue 0
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (!hw_queues()) return hipSuccess;
  ksim_stream* st = stream_of(s);
  std::shared_ptr<Cmd> last;
  {
    std::lock_guard<std::mutex> lk(g_hwq[(size_t)st->hwq]->mu);
    last = st->last;
  }
  wait_done(last);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  ksim_stream* st = stream_of(s);
  if (!hw_queues() || st->capture || !e->cmd) return hipSuccess;
  submit(st, nullptr, e->cmd);  // a barrier packet: the queue waits for the event's marker
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ksim_event;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  ksim_stream* st = stream_of(s);
  if (!hw_queues() || st->capture) return hipSuccess;
  e->cmd = submit(st, nullptr, nullptr);  // a marker
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (hw_queues()) wait_done(e->cmd);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof *p);
  strcpy(p->name, "ksim");
  strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = (int)env_long("KSIM_CUS", 4);
  p->totalGlobalMem = (size_t)1 << 36;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  *n = (int)env_long("KSIM_OCC", 2);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);  // device variables are host variables here
  return hipSuccess;
}
hipError_t hipGetLastError() {
  const hipError_t e = t_last;
  t_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "ksim error"; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capture) return hipErrorInvalidValue;
  (void)hw_queues();
  s->capture = new ksim_graph;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capture) return hipErrorInvalidValue;
  *g = s->capture;
  s->capture = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new ksim_graph(*g);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  for (auto& op : e->ops) enqueue(s, op);
  return hipSuccess;
}
