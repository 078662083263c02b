// CPU execution of liblz's kernels for tests (see shim/hip/hip_runtime.h).
// Each workgroup's work-items run as host threads; wave operations are
// rendezvous of the wave's live lanes at one call site; a lane that reaches a
// different wave operation, a barrier or its end while others of its wave
// wait in a wave operation is a divergence and stops the run.  A wait that
// does not end within the time limit stops the run as a hang.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

thread_local emu_idx threadIdx, blockIdx, blockDim, gridDim;

extern "C" {
extern uint8_t __start_lzemu_lds[] __attribute__((weak));
extern uint8_t __stop_lzemu_lds[] __attribute__((weak));
}

namespace {

constexpr int kMaxWaves = 16;
enum Op { kNone = 0, kBallot, kFirst, kLane, kShfl, kShflUp, kDpp, kWaveBar };
enum State { kRun = 0, kInWave, kInBar, kDone };

struct Group {
  std::mutex mu;
  std::condition_variable cv;
  int nthreads = 0, live = 0, bar_arrived = 0;
  std::atomic<uint64_t> bar_gen{0};
  struct Wave {
    std::condition_variable cv;        // this wave's lanes waiting in a wave operation
    int live = 0, arrived = 0;
    std::atomic<uint64_t> gen{0};
    const void* site = nullptr;
    int op = kNone, arg0 = 0, arg1 = 0, arg2 = 0, arg3 = 0;
    uint64_t nops = 0;                 // first arriving lane's operation count
    bool arg4 = false;
    uint64_t val[64], res[64];
    bool present[64];
  } wave[kMaxWaves];
  std::vector<int> state;
};

thread_local Group* g_grp = nullptr;
thread_local int g_tid = 0;
thread_local uint64_t g_nops = 0;   // wave operations this lane has reached

double g_limit_s = 120.0;

[[noreturn]] void fatal(const char* what, const void* site) {
  std::fprintf(stderr, "EMU FATAL: %s (block %u, thread %u, site %p)\n", what, blockIdx.x, threadIdx.x, site);
  Dl_info di;
  if (site && dladdr(site, &di) && di.dli_fbase)
    std::fprintf(stderr, "  site offset 0x%zx in %s\n", (size_t)((const char*)site - (const char*)di.dli_fbase),
                 di.dli_fname ? di.dli_fname : "?");
  std::fflush(stderr);
  std::abort();
}

template <class Pred>
void wait_for(std::unique_lock<std::mutex>& lk, std::condition_variable& cv, Pred p, const char* what,
              const void* site) {
  if (!cv.wait_for(lk, std::chrono::duration<double>(g_limit_s), p)) fatal(what, site);
}

// the wave's operation is complete: compute every present lane's result
void finish(Group::Wave& w, int wbase) {
  switch (w.op) {
    case kBallot: {
      uint64_t m = 0;
      for (int l = 0; l < 64; l++) if (w.present[l] && w.val[l]) m |= 1ull << l;
      for (int l = 0; l < 64; l++) w.res[l] = m;
      break;
    }
    case kFirst: {
      int f = 0;
      while (f < 64 && !w.present[f]) f++;
      for (int l = 0; l < 64; l++) w.res[l] = w.val[f];
      break;
    }
    case kLane: {
      const int src = w.arg0 & 63;
      if (!w.present[src]) { std::fprintf(stderr, "EMU FATAL: readlane of an inactive lane %d (wave at %d)\n", src, wbase); std::abort(); }
      for (int l = 0; l < 64; l++) w.res[l] = w.val[src];
      break;
    }
    case kShfl:
    case kShflUp: {
      // per lane its own source lane, recorded in res[] on arrival
      uint64_t out[64];
      for (int l = 0; l < 64; l++) {
        if (!w.present[l]) continue;
        const int src = (int)w.res[l];
        if (!w.present[src]) { std::fprintf(stderr, "EMU FATAL: shuffle from an inactive lane %d\n", src); std::abort(); }
        out[l] = w.val[src];
      }
      for (int l = 0; l < 64; l++) if (w.present[l]) w.res[l] = out[l];
      break;
    }
    case kDpp: {
      const int ctrl = w.arg0, row_mask = w.arg1, bank_mask = w.arg2;
      for (int l = 0; l < 64; l++) {
        if (!w.present[l]) continue;
        const int row = l >> 4, i = l & 15, bank = (l >> 2) & 3;
        const uint32_t old = (uint32_t)(w.val[l] >> 32);
        int src = -1;
        if (ctrl >= 0 && ctrl <= 0xFF) {                     // quad_perm
          src = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
        } else if (ctrl >= 0x111 && ctrl <= 0x11F) {         // row_shr:n
          const int n = ctrl & 0xF;
          if (i >= n) src = l - n;
        } else if (ctrl == 0x142) {                          // row_bcast:15
          if (row >= 1) src = 16 * row - 1;
        } else if (ctrl == 0x143) {                          // row_bcast:31
          if (row >= 2) src = 31;
        } else {
          std::fprintf(stderr, "EMU FATAL: unsupported DPP control 0x%x\n", ctrl);
          std::abort();
        }
        const bool write = ((row_mask >> row) & 1) && ((bank_mask >> bank) & 1);
        uint32_t r = old;
        if (write) {
          if (src >= 0) {
            if (!w.present[src]) { std::fprintf(stderr, "EMU FATAL: DPP from an inactive lane\n"); std::abort(); }
            r = (uint32_t)w.val[src];
          } else if (w.arg4) {
            r = 0;                                           // bound_ctrl: out of range reads 0
          }
        }
        w.res[l] = r;
      }
      break;
    }
    default:
      for (int l = 0; l < 64; l++) w.res[l] = 0;
  }
}

uint64_t wave_op(int op, uint64_t v, const void* site, uint64_t aux = 0, int a0 = 0, int a1 = 0, int a2 = 0,
                 int a3 = 0, bool a4 = false) {
  Group& g = *g_grp;
  const int wv = g_tid >> 6, lane = g_tid & 63;
  Group::Wave& w = g.wave[wv];
  std::unique_lock<std::mutex> lk(g.mu);
  if (w.arrived == 0) {
    // no lane of this wave may be waiting at a barrier meanwhile
    for (int l = 0; l < 64; l++) {
      const int t = 64 * wv + l;
      if (t < g.nthreads && g.state[t] == kInBar) fatal("divergent wave: a wave operation while lanes wait at a barrier", site);
    }
    w.site = site;
    w.op = op;
    w.nops = g_nops;
    w.arg0 = a0; w.arg1 = a1; w.arg2 = a2; w.arg3 = a3; w.arg4 = a4;
    for (int l = 0; l < 64; l++) w.present[l] = false;
  } else if (w.site != site || w.op != op) {
    Dl_info di;
    if (w.site && dladdr(w.site, &di) && di.dli_fbase)
      std::fprintf(stderr, "  the wave's other lanes wait at offset 0x%zx (operation %d, their %llu-th; this one %d, its %llu-th)\n",
                   (size_t)((const char*)w.site - (const char*)di.dli_fbase), w.op, (unsigned long long)w.nops, op,
                   (unsigned long long)g_nops);
    fatal("divergent wave operation (lanes of one wave at different wave operations)", site);
  }
  g_nops++;
  w.val[lane] = v;
  w.res[lane] = aux;
  w.present[lane] = true;
  g.state[g_tid] = kInWave;
  const uint64_t gen = w.gen;
  if (++w.arrived == w.live) {
    finish(w, 64 * wv);
    w.arrived = 0;
    w.gen.fetch_add(1);
    w.cv.notify_all();
  } else {
    // the other lanes are mostly runnable: yield a while before sleeping
    lk.unlock();
    for (int i = 0; i < 256 && w.gen.load() == gen; i++) std::this_thread::yield();
    lk.lock();
    wait_for(lk, w.cv, [&] { return w.gen.load() != gen; }, "hang in a wave operation", site);
  }
  g.state[g_tid] = kRun;
  return w.res[lane];
}

void run_group(dim3 grid, dim3 block, emu_body body, void* ctx, uint32_t bx) {
  Group g;
  g.nthreads = (int)(block.x * block.y * block.z);
  g.live = g.nthreads;
  g.state.assign(g.nthreads, kRun);
  for (int t = 0; t < g.nthreads; t++) g.wave[t >> 6].live++;
  if (__start_lzemu_lds && __stop_lzemu_lds)
    std::memset(__start_lzemu_lds, 0xAA, (size_t)(__stop_lzemu_lds - __start_lzemu_lds));
  std::vector<std::thread> th;
  th.reserve(g.nthreads);
  for (int t = 0; t < g.nthreads; t++) {
    th.emplace_back([&, t]() {
      threadIdx = {(uint32_t)t, 0, 0};
      blockIdx = {bx, 0, 0};
      blockDim = {block.x, block.y, block.z};
      gridDim = {grid.x, grid.y, grid.z};
      g_grp = &g;
      g_tid = t;
      body(ctx);
      std::unique_lock<std::mutex> lk(g.mu);
      Group::Wave& w = g.wave[t >> 6];
      if (w.arrived > 0) fatal("divergent wave: a lane ended while others wait in a wave operation", w.site);
      w.live--;
      g.live--;
      g.state[t] = kDone;
      if (g.bar_arrived > 0 && g.bar_arrived == g.live) {   // the others wait at a barrier
        g.bar_arrived = 0;
        for (auto& st : g.state) if (st == kInBar) st = kRun;
        g.bar_gen.fetch_add(1);
      }
      g.cv.notify_all();
    });
  }
  for (auto& x : th) x.join();
}

}  // namespace

void emu_syncthreads() {
  Group& g = *g_grp;
  std::unique_lock<std::mutex> lk(g.mu);
  const int wv = g_tid >> 6;
  if (g.wave[wv].arrived > 0) fatal("divergent wave: a barrier while lanes wait in a wave operation", nullptr);
  g.state[g_tid] = kInBar;
  const uint64_t gen = g.bar_gen.load();
  if (++g.bar_arrived == g.live) {
    g.bar_arrived = 0;
    for (auto& st : g.state) if (st == kInBar) st = kRun;   // every waiter is past the barrier
    g.bar_gen.fetch_add(1);
    g.cv.notify_all();
  } else {
    lk.unlock();
    for (int i = 0; i < 256 && g.bar_gen.load() == gen; i++) std::this_thread::yield();
    lk.lock();
    wait_for(lk, g.cv, [&] { return g.bar_gen.load() != gen; }, "hang at a workgroup barrier", nullptr);
  }
  g.state[g_tid] = kRun;
}

uint64_t emu_ballot(bool p, const void* site) { return wave_op(kBallot, p ? 1 : 0, site); }
uint32_t emu_readfirstlane(uint32_t v, const void* site) { return (uint32_t)wave_op(kFirst, v, site); }
uint32_t emu_readlane(uint32_t v, uint32_t l, const void* site) { return (uint32_t)wave_op(kLane, v, site, 0, (int)l); }
int emu_shfl(int v, int src, int width, const void* site) {
  const int lane = g_tid & 63, base = lane & ~(width - 1);
  return (int)(uint32_t)wave_op(kShfl, (uint32_t)v, site, (uint64_t)(base + (src & (width - 1))));
}
int emu_shfl_up(int v, unsigned d, int width, const void* site) {
  const int lane = g_tid & 63, i = lane & (width - 1);
  return (int)(uint32_t)wave_op(kShflUp, (uint32_t)v, site, (uint64_t)(i >= (int)d ? lane - (int)d : lane));
}
uint64_t emu_shfl64(uint64_t v, int src, int width, const void* site) {
  const int lane = g_tid & 63, base = lane & ~(width - 1);
  return wave_op(kShfl, v, site, (uint64_t)(base + (src & (width - 1))));
}
uint64_t emu_shfl_up64(uint64_t v, unsigned d, int width, const void* site) {
  const int lane = g_tid & 63, i = lane & (width - 1);
  return wave_op(kShflUp, v, site, (uint64_t)(i >= (int)d ? lane - (int)d : lane));
}
int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl, const void* site) {
  const uint64_t v = ((uint64_t)(uint32_t)old << 32) | (uint32_t)src;
  return (int)(uint32_t)wave_op(kDpp, v, site, 0, ctrl, row_mask, bank_mask, 0, bound_ctrl);
}
void emu_wave_barrier(const void* site) { wave_op(kWaveBar, 0, site); }

void emu_launch(dim3 grid, dim3 block, emu_body body, void* ctx) {
  if (const char* e = std::getenv("LZ_EMU_LIMIT_S")) g_limit_s = std::atof(e);
  for (uint32_t b = 0; b < grid.x; b++) run_group(grid, block, body, ctx, b);
}

hipError_t emu_launch_coop() { return hipErrorNotSupported; }

// ---- runtime API ----
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(d, s, n, k, nullptr); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->name, "cpu-emulation");
  p->multiProcessorCount = 2;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 2; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e ? "emulation: not supported" : "no error"; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* st) {
  *st = hipStreamCaptureStatusNone;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) { *n = 3; return hipSuccess; }
