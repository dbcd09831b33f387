// Runtime of the host-emulation build: kernel launches on a pool of host
// threads (one per thread of a block, blocks one after the other), the block
// and wave barriers, and "device" memory with guard pages.
//
// HOSTEMU_GUARD=end (default) places each allocation so that its last byte
// touches an inaccessible page (an access past the end faults at once);
// HOSTEMU_GUARD=start places the first byte right after one (an access before
// the start faults).  HOSTEMU_CUS sets the compute-unit count the library sees
// (default 2, which sizes its default grids).  A barrier that not every thread
// of a block (or lane of a wave) reaches within HOSTEMU_BARRIER_S seconds
// (default 120) aborts the process with a message.  HOSTEMU_FORK=k runs the
// blocks of a launch in up to k concurrent child processes (device memory is
// a shared mapping; host memory written by a kernel, such as a torch CPU
// tensor, is then not seen by the caller, nor is the library's static
// scratch array).
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <sys/mman.h>
#include <sys/wait.h>
#include <sched.h>
#include <unistd.h>

#include <atomic>

#include <chrono>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

thread_local hostemu::Idx threadIdx, blockIdx, blockDim, gridDim;

// bounds of the section that holds every __shared__ variable of the library
extern "C" char __start_hostemu_lds[] __attribute__((weak));
extern "C" char __stop_hostemu_lds[] __attribute__((weak));

namespace hostemu {
namespace {

double barrier_seconds() {
  const char* s = getenv("HOSTEMU_BARRIER_S");
  return s ? atof(s) : 120.0;
}

// Generation barrier of n threads with a time limit (waiters yield the CPU
// while they wait: a block has more threads than the host has cores).
struct Barrier {
  std::atomic<int> count{0};
  std::atomic<unsigned long> gen{0};
  int n = 0;
  void reset(int nthreads) {
    n = nthreads;
    count.store(0);
  }
  void wait(const char* what) {
    const unsigned long g = gen.load(std::memory_order_acquire);
    if (count.fetch_add(1, std::memory_order_acq_rel) + 1 == n) {
      count.store(0, std::memory_order_relaxed);
      gen.fetch_add(1, std::memory_order_acq_rel);
      return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const double limit = barrier_seconds();
    for (unsigned long spins = 0; gen.load(std::memory_order_acquire) == g; spins++) {
      sched_yield();
      if ((spins & 4095) == 4095 &&
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit) {
        fprintf(stderr, "hostemu: %s not reached by every thread within %.0f s (block %u, thread %u)\n", what,
                limit, blockIdx.x, threadIdx.x);
        fflush(stderr);
        abort();
      }
    }
  }
};

constexpr int kMaxThreads = 1024;

struct BlockState {
  int nthreads = 0;
  Barrier block;
  std::vector<Barrier> waves{kMaxThreads / 64};
  int flags[kMaxThreads];
  unsigned long long xch[kMaxThreads];
};
// never destroyed: the pool's threads wait on these until the process ends
BlockState& B = *new BlockState;

// Worker pool: worker i runs thread i of each block.
struct Pool {
  std::mutex m;
  std::condition_variable cv_start, cv_done;
  std::vector<std::thread> workers;
  unsigned long job = 0;
  int running = 0;
  int nthreads = 0;
  dim3 grid, block, bidx;
  void (*body)(void*) = nullptr;
  void* ctx = nullptr;

  void ensure(int n) {
    while ((int)workers.size() < n) {
      const int id = (int)workers.size();
      workers.emplace_back([this, id] { work(id); });
      workers.back().detach();
    }
  }
  void work(int id) {
    unsigned long seen = 0;
    for (;;) {
      void (*f)(void*);
      void* c;
      {
        std::unique_lock<std::mutex> lk(m);
        cv_start.wait(lk, [&] { return job != seen; });
        seen = job;
        if (id >= nthreads) continue;
        f = body;
        c = ctx;
        const unsigned bx = block.x, by = block.y;
        threadIdx.x = id % bx;
        threadIdx.y = (id / bx) % by;
        threadIdx.z = id / (bx * by);
        blockIdx.x = bidx.x;
        blockIdx.y = bidx.y;
        blockIdx.z = bidx.z;
        blockDim.x = block.x;
        blockDim.y = block.y;
        blockDim.z = block.z;
        gridDim.x = grid.x;
        gridDim.y = grid.y;
        gridDim.z = grid.z;
      }
      f(c);
      {
        std::lock_guard<std::mutex> lk(m);
        if (--running == 0) cv_done.notify_all();
      }
    }
  }
  void run_block(dim3 g, dim3 b, dim3 bi, void (*f)(void*), void* c, int n) {
    // 0x7F bytes: an int read before it is written is a large index and a
    // double is 3.4e304, so a use of block memory left from before shows
    if (__start_hostemu_lds && __stop_hostemu_lds > __start_hostemu_lds)
      memset(__start_hostemu_lds, 0x7F, (size_t)(__stop_hostemu_lds - __start_hostemu_lds));
    std::unique_lock<std::mutex> lk(m);
    grid = g;
    block = b;
    bidx = bi;
    body = f;
    ctx = c;
    nthreads = n;
    running = n;
    job++;
    cv_start.notify_all();
    cv_done.wait(lk, [&] { return running == 0; });
  }
};
Pool& pool = *new Pool;
std::mutex& launch_mutex = *new std::mutex;

int thread_linear() { return (int)(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z)); }

}  // namespace

int lane_index() { return thread_linear() % 64; }
int block_threads() { return B.nthreads; }

void block_barrier() { B.block.wait("__syncthreads"); }

int block_or(int p) {
  const int t = thread_linear();
  B.flags[t] = p;
  B.block.wait("__syncthreads_or");
  int r = 0;
  for (int i = 0; i < B.nthreads; i++) r |= B.flags[i] != 0;
  B.block.wait("__syncthreads_or");
  return r;
}

unsigned long long wave_ballot(int p) {
  const int t = thread_linear(), w = t / 64;
  B.flags[t] = p;
  B.waves[w].wait("__ballot");
  unsigned long long m = 0;
  const int lanes = std::min(64, B.nthreads - 64 * w);
  for (int l = 0; l < lanes; l++)
    if (B.flags[64 * w + l]) m |= 1ull << l;
  B.waves[w].wait("__ballot");
  return m;
}

unsigned long long wave_exchange(unsigned long long v, int src_lane) {
  const int t = thread_linear(), w = t / 64;
  B.xch[t] = v;
  B.waves[w].wait("wave exchange");
  const int lanes = std::min(64, B.nthreads - 64 * w);
  const unsigned long long r = (src_lane >= 0 && src_lane < lanes) ? B.xch[64 * w + src_lane] : v;
  B.waves[w].wait("wave exchange");
  return r;
}

void wave_gather(unsigned long long v, unsigned long long* all64) {
  const int t = thread_linear(), w = t / 64;
  B.xch[t] = v;
  B.waves[w].wait("wave exchange");
  const int lanes = std::min(64, B.nthreads - 64 * w);
  for (int l = 0; l < 64; l++) all64[l] = l < lanes ? B.xch[64 * w + l] : 0ull;
  B.waves[w].wait("wave exchange");
}

int fork_width() {
  const char* s = getenv("HOSTEMU_FORK");
  return s ? atoi(s) : 0;
}

void run_kernel(dim3 grid, dim3 block, void (*body)(void*), void* ctx) {
  std::lock_guard<std::mutex> lk(launch_mutex);
  const int n = (int)(block.x * block.y * block.z);
  if (n <= 0 || n > kMaxThreads) unsupported("block size");
  const long nblocks = (long)grid.x * grid.y * grid.z;
  const int width = fork_width();
  if (width > 1 && nblocks > 1) {
    // blocks in concurrent child processes, each with its own "LDS" (its
    // copy of the static block memory) and its own thread pool; device
    // memory is shared (see hipMalloc)
    fflush(stdout);
    fflush(stderr);
    int active = 0, failed = 0;
    auto reap = [&](int options) {
      int st = 0;
      pid_t pid = waitpid(-1, &st, options);
      if (pid > 0) {
        active--;
        if (!WIFEXITED(st) || WEXITSTATUS(st) != 0) {
          fprintf(stderr, "hostemu: a block process ended abnormally (%s %d)\n",
                  WIFSIGNALED(st) ? "signal" : "exit status", WIFSIGNALED(st) ? WTERMSIG(st) : WEXITSTATUS(st));
          failed++;
        }
      }
      return pid;
    };
    for (long b = 0; b < nblocks; b++) {
      while (active >= width) reap(0);
      pid_t pid = fork();
      if (pid < 0) unsupported("fork");
      if (pid == 0) {
        Pool* fresh = new Pool;  // the parent's pool threads do not exist here
        fresh->ensure(n);
        B.nthreads = n;
        B.block.reset(n);
        for (int w = 0; w * 64 < n; w++) B.waves[w].reset(std::min(64, n - 64 * w));
        const unsigned x = (unsigned)(b % grid.x), y = (unsigned)((b / grid.x) % grid.y),
                       z = (unsigned)(b / ((long)grid.x * grid.y));
        fresh->run_block(grid, block, dim3(x, y, z), body, ctx, n);
        fflush(stdout);
        fflush(stderr);
        _exit(0);
      }
      active++;
    }
    while (active > 0) reap(0);
    if (failed) abort();
    return;
  }
  pool.ensure(n);
  B.nthreads = n;
  B.block.reset(n);
  for (int w = 0; w * 64 < n; w++) B.waves[w].reset(std::min(64, n - 64 * w));
  for (unsigned z = 0; z < grid.z; z++)
    for (unsigned y = 0; y < grid.y; y++)
      for (unsigned x = 0; x < grid.x; x++) pool.run_block(grid, block, dim3(x, y, z), body, ctx, n);
}

void unsupported(const char* what) {
  fprintf(stderr, "hostemu: unsupported: %s\n", what);
  fflush(stderr);
  abort();
}

}  // namespace hostemu

// --- memory with guard pages -------------------------------------------------------
namespace {
struct Mapping {
  void* base;
  size_t len;
};
std::mutex mem_mutex;
std::map<void*, Mapping> mappings;
hipError_t last_error = hipSuccess;

bool guard_at_start() {
  const char* s = getenv("HOSTEMU_GUARD");
  return s && s[0] == 's';
}
}  // namespace

hipError_t hipMalloc(void** p, size_t n) {
  const size_t page = (size_t)sysconf(_SC_PAGESIZE);
  const size_t sz = std::max<size_t>((n + 15) & ~(size_t)15, 16);
  const size_t body = (sz + page - 1) / page * page;
  const size_t len = body + 2 * page;
  void* base = mmap(nullptr, len, PROT_NONE, MAP_SHARED | MAP_ANONYMOUS, -1, 0);
  if (base == MAP_FAILED) return last_error = hipErrorOutOfMemory;
  char* b = (char*)base + page;
  if (mprotect(b, body, PROT_READ | PROT_WRITE) != 0) {
    munmap(base, len);
    return last_error = hipErrorOutOfMemory;
  }
  char* q = guard_at_start() ? b : b + body - sz;
  memset(q, 0xA5, sz);  // not zero: reads of memory never written show up
  std::lock_guard<std::mutex> lk(mem_mutex);
  mappings[q] = Mapping{base, len};
  *p = q;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::mutex> lk(mem_mutex);
  auto it = mappings.find(p);
  if (it == mappings.end()) {
    fprintf(stderr, "hostemu: hipFree of a pointer hipMalloc did not return\n");
    abort();
  }
  munmap(it->second.base, it->second.len);
  mappings.erase(it);
  return hipSuccess;
}

hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemset(void* p, int v, size_t n) {
  if (n) memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { return hipMemset(p, v, n); }
hipError_t hipGetLastError() {
  hipError_t e = last_error;
  last_error = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "host emulation error"; }
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof(*p));
  strcpy(p->name, "host emulation");
  const char* s = getenv("HOSTEMU_CUS");
  p->multiProcessorCount = s ? atoi(s) : 2;
  p->totalGlobalMem = (size_t)16 << 30;
  p->warpSize = 64;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char[1]);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete[] reinterpret_cast<char*>(s);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* st) {
  *st = hipStreamCaptureStatusNone;
  return hipSuccess;
}
// graphs are not emulated
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = nullptr;
  return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

struct ihipEvent_t {
  std::chrono::steady_clock::time_point t;
};
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->t = std::chrono::steady_clock::now();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)std::chrono::duration<double, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
