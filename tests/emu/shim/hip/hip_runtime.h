// CPU stand-in for the HIP device language used by liblz's kernels (test
// harness only).  Every work-item runs on a host thread of its own; a
// workgroup's threads run together, workgroups one after another.  Wave
// operations (ballot, readfirstlane, readlane, shuffles, DPP moves, wave
// barriers, wavefront fences) are rendezvous of the wave's 64 lanes: every
// live lane of the wave must reach the same call site, else the harness stops
// with "divergent wave operation" -- on gfx950 such an operation would see only
// the lanes active there, so the kernel's results would depend on how the
// compiler structured the branch.  LDS (__shared__) is poisoned before every
// workgroup.
#pragma once
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <tuple>
#include <utility>

#include "hip_runtime_api.h"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static __attribute__((section("lzemu_lds")))
#define HIP_SYMBOL(x) (&(x))
#define __align__(n) __attribute__((aligned(n)))
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4

struct uint4 { uint32_t x, y, z, w; };
struct uint2 { uint32_t x, y; };
struct dim3 {
  uint32_t x, y, z;
  dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct emu_idx { uint32_t x, y, z; };
extern thread_local emu_idx threadIdx, blockIdx;
extern thread_local emu_idx blockDim, gridDim;

// ---- wave and workgroup operations (emu.cpp) ----
void emu_syncthreads();
uint64_t emu_ballot(bool p, const void* site);
uint32_t emu_readfirstlane(uint32_t v, const void* site);
uint32_t emu_readlane(uint32_t v, uint32_t lane, const void* site);
int emu_shfl(int v, int src, int width, const void* site);
int emu_shfl_up(int v, unsigned d, int width, const void* site);
int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl, const void* site);
void emu_wave_barrier(const void* site);

#define EMU_SITE (__builtin_return_address(0))
__attribute__((noinline)) inline void __syncthreads() { emu_syncthreads(); }
__attribute__((noinline)) inline uint64_t __ballot(int p) { return emu_ballot(p != 0, EMU_SITE); }
__attribute__((noinline)) inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) {
  return emu_readfirstlane(v, EMU_SITE);
}
__attribute__((noinline)) inline uint32_t __builtin_amdgcn_readlane(uint32_t v, uint32_t l) {
  return emu_readlane(v, l, EMU_SITE);
}
__attribute__((noinline)) inline int __shfl(int v, int src, int width = 64) { return emu_shfl(v, src, width, EMU_SITE); }
__attribute__((noinline)) inline unsigned __shfl(unsigned v, int src, int width = 64) {
  return (unsigned)emu_shfl((int)v, src, width, EMU_SITE);
}
__attribute__((noinline)) inline int __shfl_up(int v, unsigned d, int width = 64) {
  return emu_shfl_up(v, d, width, EMU_SITE);
}
__attribute__((noinline)) inline unsigned __shfl_up(unsigned v, unsigned d, int width = 64) {
  return (unsigned)emu_shfl_up((int)v, d, width, EMU_SITE);
}
uint64_t emu_shfl64(uint64_t v, int src, int width, const void* site);
uint64_t emu_shfl_up64(uint64_t v, unsigned d, int width, const void* site);
__attribute__((noinline)) inline unsigned long __shfl(unsigned long v, int src, int width = 64) {
  return (unsigned long)emu_shfl64(v, src, width, EMU_SITE);
}
__attribute__((noinline)) inline unsigned long __shfl_up(unsigned long v, unsigned d, int width = 64) {
  return (unsigned long)emu_shfl_up64(v, d, width, EMU_SITE);
}
__attribute__((noinline)) inline unsigned long long __shfl(unsigned long long v, int src, int width = 64) {
  return emu_shfl64(v, src, width, EMU_SITE);
}
__attribute__((noinline)) inline unsigned long long __shfl_up(unsigned long long v, unsigned d, int width = 64) {
  return emu_shfl_up64(v, d, width, EMU_SITE);
}
__attribute__((noinline)) inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int rm, int bm, bool bc) {
  return emu_update_dpp(old, src, ctrl, rm, bm, bc, EMU_SITE);
}
__attribute__((noinline)) inline int __builtin_amdgcn_mov_dpp(int src, int ctrl, int rm, int bm, bool bc) {
  // identity quad_perm with every row and bank written: each lane reads its
  // own register, so it is lane-local and legal in divergent code
  if (ctrl == 0xE4 && rm == 0xF && bm == 0xF) return src;
  return emu_update_dpp(0, src, ctrl, rm, bm, bc, EMU_SITE);
}
__attribute__((noinline)) inline void __builtin_amdgcn_wave_barrier() { emu_wave_barrier(EMU_SITE); }
inline void __builtin_amdgcn_sched_barrier(int) { }
// global_load_lds: lane k's `size` bytes from src land at dst + off + size k
// (dst is the wave's uniform LDS address); the copy is done at once, so the
// wait that the device needs before reading is a no-op here
inline void __builtin_amdgcn_global_load_lds(const void* src, void* dst, unsigned size, int off, int) {
  std::memcpy(static_cast<char*>(dst) + off + size * (threadIdx.x & 63u), src, size);
}
inline void __builtin_amdgcn_s_waitcnt(int) { }
inline void __builtin_amdgcn_s_setprio(int) { }
__attribute__((noinline)) inline void __builtin_amdgcn_fence(int order, const char* scope) {
  if (scope && !std::strcmp(scope, "wavefront")) emu_wave_barrier(EMU_SITE);
  else std::atomic_thread_fence(std::memory_order_seq_cst);
  (void)order;
}

inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t base) {
  const uint32_t l = threadIdx.x & 63;
  return base + (uint32_t)__builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1u)));
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t base) {
  const uint32_t l = threadIdx.x & 63;
  return base + (l < 32 ? 0u : (uint32_t)__builtin_popcount(m & ((l == 32 ? 0u : (1u << (l - 32)) - 1u))));
}
inline uint32_t __builtin_amdgcn_alignbyte(uint32_t hi, uint32_t lo, uint32_t s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * (s & 3)));
}
inline void __builtin_amdgcn_s_sleep(int) { }
inline uint32_t __umul24(uint32_t a, uint32_t b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }

// atomics: host atomics (work-items of a workgroup run concurrently)
template <class T> inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T __hip_atomic_load(T* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T> inline T __hip_atomic_load(const T* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T, class U> inline void __hip_atomic_store(T* p, U v, int, int) {
  __atomic_store_n(p, (T)v, __ATOMIC_SEQ_CST);
}
template <class T, class U> inline T __hip_atomic_fetch_add(T* p, U v, int, int) {
  return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST);
}
template <class T, class U> inline T __hip_atomic_fetch_or(T* p, U v, int, int) {
  return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST);
}
template <class T, class U> inline T __hip_atomic_fetch_max(T* p, U v, int, int) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (cur < (T)v && !__atomic_compare_exchange_n(p, &cur, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}

// device min/max: one type, as the HIP headers' integer overloads
template <class T> inline T min(T a, T b) { return b < a ? b : a; }
template <class T> inline T max(T a, T b) { return a < b ? b : a; }

// ---- launches (emu.cpp) ----
typedef void (*emu_body)(void*);
void emu_launch(dim3 grid, dim3 block, emu_body body, void* ctx);
hipError_t emu_launch_coop();

template <class... P, class... A>
inline void emu_launch_kernel(void (*k)(P...), dim3 grid, dim3 block, A&&... a) {
  auto args = std::make_tuple(static_cast<P>(a)...);
  struct Ctx { void (*k)(P...); decltype(args)* t; } c{k, &args};
  emu_launch(grid, block, [](void* p) {
    auto* cc = static_cast<Ctx*>(p);
    std::apply(cc->k, *cc->t);
  }, &c);
}
#define hipLaunchKernelGGL(k, grid, block, smem, stream, ...) emu_launch_kernel(k, dim3(grid), dim3(block), ##__VA_ARGS__)
inline hipError_t hipLaunchCooperativeKernel(const void*, dim3, dim3, void**, size_t, hipStream_t) {
  return emu_launch_coop();
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
