// Device decoder for container format v1 on gfx950 (CDNA4, wave64).
//
// One workgroup of 256 threads (4 waves) decodes one block at a time:
//   1. stage the rANS bodies of the command (CMD), match-length (MLEN) and
//      offset (OFF) streams in LDS; waves 0..2 decode one stream each;
//   2. block-wide exclusive scans turn literal-run and match lengths into
//      literal and output positions (command placement);
//   3. the literal stream's 64-lane groups are decoded by one wave each and
//      every literal is written straight to its output position in an LDS tile;
//   4. matches whose source lies wholly in earlier blocks are copied in
//      parallel; then the remaining matches are copied in order, a chunk of
//      min(period, 64) bytes at a time, which reproduces the byte-sequential
//      overlap rule out[p+k] = out[OF+k];
//   5. the tile is written to HBM with 16-byte stores and, in the persistent
//      kernel, the block's completion flag is released.
// Blocks are taken in dependency-level order ("wavefront" order, paper:
// Background section), either one launch per level or one persistent launch
// whose workgroups take tickets and wait on the flags of a block's
// dependencies.  No MFMA: nothing here is a contraction.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lz_internal.h"

namespace {

constexpr int kWG = 256;
constexpr int kWaves = kWG / 64;
constexpr uint32_t kB = 1u << kMaxBlockLog2;      // largest block: 16 KiB tile
constexpr uint32_t kMaxSeq = 1025;                // B/m + 1 for B = 16 KiB, m = 16
constexpr uint32_t kLutLit = 1u << kMaxPLit;      // 4096 entries
constexpr uint32_t kLutSeq = 1u << kMaxPSeq;      // 1024 entries per small table
constexpr uint32_t kLutWords = kLutLit + 3 * kLutSeq;
constexpr uint32_t kStage = kB;                   // staging bytes (rANS bodies)
constexpr uint32_t kL = 1u << 16;                 // rANS state lower bound

__device__ __forceinline__ uint32_t lut_base(int kind) {
  return kind == kLit ? 0u : kLutLit + (uint32_t)(kind - 1) * kLutSeq;
}

struct Smem {
  uint32_t lut[kLutWords];
  uint8_t tile[kB];
  alignas(16) uint8_t stage[kStage];
  uint64_t of[kMaxSeq];
  uint16_t ll[kMaxSeq + 1];
  uint16_t ml[kMaxSeq + 1];
  uint16_t lit[kMaxSeq + 1];   // exclusive scan of LL; [ns] = n_lit
  uint16_t out[kMaxSeq + 1];   // exclusive scan of LL + ML; [ns] = block length
  uint32_t scan[kWaves];
  uint32_t hdr[4][6];          // per stream: mode, csym, K, n, nw, body_len
  uint32_t body_off[4];        // byte offset of each body inside the block payload
  uint32_t item, err, nint;
  uint16_t intl[kMaxSeq];      // indices of in-block / mixed-source matches
};

struct DevArgs {
  const uint8_t* arc;
  uint64_t n, off_dir, off_dep_ptr, off_dep_idx, off_payload;
  uint32_t bl, w, m, lit_lanes, seq_lanes;
  uint32_t P[4];
  const uint32_t* lut;      // workspace LUT images
  const uint32_t* queue;    // block ids in level order
  const uint32_t* qptr;     // device count / offsets (see launch)
  uint32_t q_begin, q_end;  // static slice (per-level launch) when qcount == null
  const uint32_t* qcount;   // device-side queue length (request mode) or null
  uint8_t* out;             // whole-file output base (direct mode)
  const uint64_t* addr;     // per-block device address (request mode) or null
  uint32_t* flags;
  uint32_t* ctl;
  uint32_t persistent;
  uint32_t spin_limit;
};

__device__ __forceinline__ uint32_t ld32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
__device__ __forceinline__ uint64_t ld64(const uint8_t* p) {
  return (uint64_t)ld32(p) | ((uint64_t)ld32(p + 4) << 32);
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void latch(uint32_t* ctl, uint32_t bits) {
  __hip_atomic_fetch_or(ctl + kCtlStatus, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decode the symbols of one 64-lane group g of a rANS stream (one wave).
// body: LDS copy of the record body (states, group word counts, words).
// Returns true if the group ends with every state at 2^16 and every word read.
template <class Out>
__device__ bool rans_group(const uint8_t* body, uint32_t K, uint32_t n, uint32_t g,
                           const uint32_t* lut, uint32_t P, Out&& out) {
  const uint32_t lane = lane_id();
  const uint32_t G = (K + 63) >> 6;
  const uint32_t k = (g << 6) + lane;
  const bool lane_ok = k < K;
  const uint32_t* st = reinterpret_cast<const uint32_t*>(body);
  const uint32_t* gw = st + K;
  uint32_t woff = 0;
  for (uint32_t q = 0; q < g; q++) woff += gw[q];
  const uint32_t nwg = gw[g];
  const uint16_t* W = reinterpret_cast<const uint16_t*>(gw + G) + woff;
  uint32_t x = lane_ok ? st[k] : kL;
  bool ok = x >= kL;
  uint32_t pos = 0;
  const uint32_t rounds = (n + K - 1) / K;
  const uint32_t mask = (1u << P) - 1;
  uint32_t i = k;
  for (uint32_t r = 0; r < rounds; r++, i += K) {
    const bool act = lane_ok && i < n;
    if (act) {
      const uint32_t e = lut[x & mask];
      x = __umul24((e >> 8) & 0xFFFu, x >> P) + (e >> 20);
      out(i, e & 0xFFu);
    }
    const bool need = act && x < kL;
    const uint64_t bal = __ballot(need);
    if (need) {
      const uint32_t idx = pos + mbcnt(bal);
      const bool in = idx < nwg;
      ok = ok && in;
      x = (x << 16) | (in ? (uint32_t)W[idx] : 0u);
    }
    pos += (uint32_t)__popcll(bal);
  }
  ok = ok && (!lane_ok || x == kL) && pos == nwg;
  return __ballot(!ok) == 0;
}

// Source byte at absolute position a for a match copy: direct mode reads the
// whole-file output; request mode goes through the per-block address table.
__device__ __forceinline__ uint32_t src_byte(const DevArgs& A, uint64_t a, bool& bad) {
  if (!A.addr) return A.out[a];
  const uint64_t base = A.addr[a >> A.bl];
  if (!base) { bad = true; return 0; }
  return reinterpret_cast<const uint8_t*>(base)[a & ((1ull << A.bl) - 1)];
}

// Block-wide exclusive scan of v (one value per thread); returns the prefix
// and writes the total to *total.
__device__ uint32_t block_scan(Smem& S, uint32_t v, uint32_t* total) {
  const uint32_t t = threadIdx.x, lane = lane_id(), wv = t >> 6;
  uint32_t incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= (uint32_t)d) incl += y;
  }
  if (lane == 63) S.scan[wv] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int q = 0; q < kWaves; q++) {
    uint32_t s = S.scan[q];
    if (q < (int)wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// Parse the 4 stream records of a block; fills S.hdr / S.body_off.  Thread 0.
__device__ bool parse_streams(Smem& S, const uint8_t* pay, uint32_t plen, uint32_t ns,
                              uint32_t nlit, const DevArgs& A) {
  static constexpr int order[4] = {kCmd, kMlen, kOff, kLit};
  uint32_t off = 0;
  for (int q = 0; q < 4; q++) {
    const int kind = order[q];
    if (off + 16 > plen) return false;
    const uint8_t* h = pay + off;
    const uint32_t mode = h[0], csym = h[1], K = (uint32_t)h[2] | ((uint32_t)h[3] << 8);
    const uint32_t n = ld32(h + 4), nw = ld32(h + 8), bl = ld32(h + 12);
    const uint32_t want = kind == kLit ? nlit : (kind == kOff ? A.w * ns : 2 * ns);
    if (n != want) return false;
    const uint32_t body = off + 16;
    const uint32_t maxK = kind == kLit ? A.lit_lanes : A.seq_lanes;
    switch (mode) {
      case kModeEmpty: if (n != 0 || bl != 0) return false; break;
      case kModeConst: if (n == 0 || bl != 0) return false; break;
      case kModeRaw: if (bl != n || body + bl > plen) return false; break;
      case kModeRans: {
        const uint32_t G = (K + 63) >> 6;
        if (K < 1 || K > maxK || n == 0 || body + bl > plen) return false;
        if ((uint64_t)bl != 4ull * K + 4ull * G + 2ull * nw) return false;
        if (bl > kStage) return false;
        uint64_t sum = 0;     // per-group word counts must add up to n_words
        for (uint32_t g = 0; g < G; g++) sum += ld32(pay + body + 4 * K + 4 * g);
        if (sum != nw) return false;
        break;
      }
      default: return false;
    }
    uint32_t* hd = S.hdr[kind];
    hd[0] = mode; hd[1] = csym; hd[2] = K; hd[3] = n; hd[4] = nw; hd[5] = bl;
    S.body_off[kind] = body;
    off = body + ((bl + 15u) & ~15u);
  }
  return true;
}

// Copy rANS bodies of the given kinds from global to consecutive 16-byte
// aligned LDS staging offsets; returns the staging offset of each.
__device__ void stage_bodies(Smem& S, const uint8_t* pay, const int* kinds, int nk, uint32_t* soff) {
  uint32_t o = 0;
  for (int q = 0; q < nk; q++) {
    soff[q] = o;
    if (S.hdr[kinds[q]][0] == kModeRans) o += (S.hdr[kinds[q]][5] + 15u) & ~15u;
  }
  for (int q = 0; q < nk; q++) {
    const int kind = kinds[q];
    if (S.hdr[kind][0] != kModeRans) continue;
    const uint32_t bl = S.hdr[kind][5];
    const uint4* src = reinterpret_cast<const uint4*>(pay + S.body_off[kind]);
    uint4* dst = reinterpret_cast<uint4*>(S.stage + soff[q]);
    for (uint32_t c = threadIdx.x; c < (bl + 15u) >> 4; c += kWG) dst[c] = src[c];
  }
}

// Decode one whole block b into the LDS tile and store it; returns false on a
// corrupt block (status already latched).
__device__ void decode_block(Smem& S, const DevArgs& A, uint32_t b) {
  const uint32_t t = threadIdx.x, wv = t >> 6, lane = lane_id();
  const uint64_t B = 1ull << A.bl;
  const uint64_t sb = (uint64_t)b << A.bl;
  const uint32_t blen = (uint32_t)((sb + B <= A.n) ? B : A.n - sb);
  const uint8_t* de = A.arc + A.off_dir + (uint64_t)b * kDirEntry;
  const uint64_t poff = ld64(de);
  const uint32_t plen = ld32(de + 8), ns = ld32(de + 12), nlit = ld32(de + 16);
  const uint8_t* pay = A.arc + A.off_payload + poff;

  if (t == 0) {
    bool ok = ns >= 1 && ns <= kMaxSeq && nlit <= blen && ((poff & 15) == 0);
    ok = ok && parse_streams(S, pay, plen, ns, nlit, A);
    S.err = ok ? 0u : 1u;
  }
  __syncthreads();
  if (S.err) { if (t == 0) latch(A.ctl, kStCorrupt); return; }

  // ---- stage 1: small streams
  static constexpr int small[3] = {kCmd, kMlen, kOff};
  uint32_t soff[3];
  stage_bodies(S, pay, small, 3, soff);
  for (uint32_t j = t; j < ns; j += kWG) S.of[j] = 0;
  __syncthreads();
  bool ok = true;
  if (wv < 3) {
    const int kind = small[wv];
    const uint32_t* hd = S.hdr[kind];
    const uint32_t mode = hd[0], n = hd[3];
    uint8_t* dstb = kind == kCmd ? reinterpret_cast<uint8_t*>(S.ll)
                  : kind == kMlen ? reinterpret_cast<uint8_t*>(S.ml)
                                  : reinterpret_cast<uint8_t*>(S.of);
    const uint32_t stride = kind == kOff ? 8u : 2u;
    auto put = [&](uint32_t i, uint32_t s) {
      uint32_t plane = 0, idx = i;
      while (idx >= ns) { idx -= ns; plane++; }
      dstb[idx * stride + plane] = (uint8_t)s;
    };
    if (mode == kModeRans) {
      ok = rans_group(S.stage + soff[wv], hd[2], n, 0, S.lut + lut_base(kind), A.P[kind], put);
    } else if (mode == kModeRaw) {
      const uint8_t* src = pay + S.body_off[kind];
      for (uint32_t i = lane; i < n; i += 64) put(i, src[i]);
    } else if (mode == kModeConst) {
      for (uint32_t i = lane; i < n; i += 64) put(i, hd[1]);
    }
  }
  if (!ok && lane == 0) S.err = 1;
  __syncthreads();
  if (S.err) { if (t == 0) latch(A.ctl, kStCorrupt); return; }

  // ---- stage 2: command placement (exclusive scans of LL and LL + ML)
  {
    const uint32_t per = (ns + kWG - 1) / kWG;
    const uint32_t j0 = t * per, j1 = min(ns, j0 + per);
    uint32_t sl = 0, so = 0;
    for (uint32_t j = j0; j < j1; j++) { sl += S.ll[j]; so += S.ll[j] + S.ml[j]; }
    uint32_t tl, to;
    uint32_t bl_ = block_scan(S, sl, &tl);
    uint32_t bo = block_scan(S, so, &to);
    bool bad = false;
    for (uint32_t j = j0; j < j1; j++) {
      S.lit[j] = (uint16_t)bl_;
      S.out[j] = (uint16_t)bo;
      const uint32_t L = S.ll[j], M = S.ml[j];
      const uint64_t of = S.of[j];
      const uint64_t dst = sb + bo + L;
      if (M == 0) bad |= (j != ns - 1) || of != 0;
      else bad |= M < A.m || of >= dst;
      bl_ += L;
      bo += L + M;
    }
    if (t == 0) { S.lit[ns] = (uint16_t)min(tl, 65535u); S.out[ns] = (uint16_t)min(to, 65535u); }
    if (tl != nlit || to != blen) bad = true;
    if (bad) S.err = 1;
    if (t == 0) S.nint = 0;
  }
  __syncthreads();
  if (S.err) { if (t == 0) latch(A.ctl, kStCorrupt); return; }

  // ---- stage 3: literals straight into the tile
  {
    static constexpr int litk[1] = {kLit};
    const uint32_t* hd = S.hdr[kLit];
    const uint32_t mode = hd[0], n = hd[3];
    uint32_t so1[1];
    stage_bodies(S, pay, litk, 1, so1);
    __syncthreads();
    uint32_t j = 0;   // per-lane current sequence (monotone in i)
    auto place = [&](uint32_t i, uint32_t s) {
      while (i >= S.lit[j + 1]) j++;
      S.tile[S.out[j] + (i - S.lit[j])] = (uint8_t)s;
    };
    bool okl = true;
    if (mode == kModeRans) {
      const uint32_t G = (hd[2] + 63) >> 6;
      for (uint32_t g = wv; g < G; g += kWaves)
        okl = okl && rans_group(S.stage, hd[2], n, g, S.lut + lut_base(kLit), A.P[kLit], place);
    } else if (mode == kModeRaw) {
      const uint8_t* src = pay + S.body_off[kLit];
      for (uint32_t i = t; i < n; i += kWG) place(i, src[i]);
    } else if (mode == kModeConst) {
      for (uint32_t i = t; i < n; i += kWG) place(i, hd[1]);
    }
    if (!okl && lane == 0) S.err = 1;
    // classify matches: wholly external ones are copied now, in parallel
    bool bad = false;
    for (uint32_t q = wv; q < ns; q += kWaves) {
      const uint32_t M = S.ml[q];
      if (!M) continue;
      const uint64_t of = S.of[q];
      if (of + M <= sb) {
        const uint32_t d0 = S.out[q] + S.ll[q];
        for (uint32_t k = lane; k < M; k += 64) S.tile[d0 + k] = (uint8_t)src_byte(A, of + k, bad);
      } else if (lane == 0) {
        S.intl[atomicAdd(&S.nint, 1u)] = q;
      }
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) { if (t == 0) latch(A.ctl, kStCorrupt); return; }

  // ---- stage 4: in-block / mixed-source matches in sequence order (wave 0)
  if (wv == 0 && S.nint) {
    // order the (few) collected matches by sequence index: insertion sort
    const uint32_t cnt = S.nint;
    if (lane == 0)
      for (uint32_t a = 1; a < cnt; a++) {
        uint32_t v = S.intl[a], c = a;
        while (c > 0 && S.intl[c - 1] > v) { S.intl[c] = S.intl[c - 1]; c--; }
        S.intl[c] = v;
      }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    bool bad = false;
    for (uint32_t a = 0; a < cnt; a++) {
      const uint32_t q = S.intl[a];
      const uint32_t M = S.ml[q];
      const uint32_t d0 = S.out[q] + S.ll[q];
      const uint64_t of = S.of[q];
      const uint64_t dabs = sb + d0;
      const uint32_t step = (dabs - of) < 64 ? (uint32_t)(dabs - of) : 64u;
      for (uint32_t c = 0; c < M; c += step) {
        const uint32_t k = c + lane;
        if (lane < step && k < M) {
          const uint64_t s = of + k;
          const uint32_t v = s >= sb ? (uint32_t)S.tile[s - sb] : src_byte(A, s, bad);
          S.tile[d0 + k] = (uint8_t)v;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) { if (t == 0) latch(A.ctl, kStCorrupt); return; }

  // ---- stage 5: tile -> HBM, 16-byte stores
  uint8_t* dst = A.addr ? reinterpret_cast<uint8_t*>(A.addr[b]) : A.out + sb;
  if (dst) {
    const uint32_t full = blen >> 4;
    const uint4* s4 = reinterpret_cast<const uint4*>(S.tile);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (uint32_t c = t; c < full; c += kWG) d4[c] = s4[c];
    for (uint32_t c = (full << 4) + t; c < blen; c += kWG) dst[c] = S.tile[c];
  }
}

__device__ void load_luts(Smem& S, const uint32_t* lut) {
  const uint4* s = reinterpret_cast<const uint4*>(lut);
  uint4* d = reinterpret_cast<uint4*>(S.lut);
  for (uint32_t c = threadIdx.x; c < kLutWords / 4; c += kWG) d[c] = s[c];
}

__global__ void __launch_bounds__(kWG) k_decode(DevArgs A) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  Smem& S = *reinterpret_cast<Smem*>(smem_raw);
  const uint32_t t = threadIdx.x;
  load_luts(S, A.lut);
  __syncthreads();
  const uint32_t epoch = __hip_atomic_load(A.ctl + kCtlEpoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t qb = A.q_begin, qe = A.q_end;
  if (A.qptr) {            // request mode: slice bounds read on the device
    qb = A.qptr[A.q_begin];
    qe = A.qptr[A.q_end];
  }
  if (!A.persistent) {
    for (uint32_t it = qb + blockIdx.x; it < qe; it += gridDim.x) {
      decode_block(S, A, A.queue[it]);
      __syncthreads();
    }
    return;
  }
  for (;;) {
    if (t == 0) S.item = qb + atomicAdd(A.ctl + kCtlTicket, 1u);
    __syncthreads();
    const uint32_t it = S.item;
    __syncthreads();
    if (it >= qe) break;
    const uint32_t b = A.queue[it];
    // wait for every dependency's completion flag (acquire)
    const uint64_t d0 = ld64(A.arc + A.off_dep_ptr + 8ull * b);
    const uint64_t d1 = ld64(A.arc + A.off_dep_ptr + 8ull * (b + 1));
    for (uint64_t k = d0 + t; k < d1; k += kWG) {
      const uint32_t d = ld32(A.arc + A.off_dep_idx + 4 * k);
      uint32_t spins = 0;
      while (__hip_atomic_load(A.flags + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > A.spin_limit) { latch(A.ctl, kStWatchdog); break; }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    decode_block(S, A, b);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (t == 0) __hip_atomic_store(A.flags + b, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- setup kernels ---------------------------------------------------------

// Packed decode entry of slot u: symbol | f << 8 | (u - c_s) << 20, for the
// four tables (LIT with 2^P_LIT slots, the others with 2^P slots each).
__global__ void k_build_lut(const uint8_t* arc, uint64_t off_tables, uint32_t p0, uint32_t p1,
                            uint32_t p2, uint32_t p3, uint32_t* lut) {
  __shared__ uint32_t cum[257];
  __shared__ uint32_t fr[256];
  const int kind = blockIdx.x;
  const uint32_t P = kind == 0 ? p0 : kind == 1 ? p1 : kind == 2 ? p2 : p3;
  const uint8_t* tab = arc + off_tables + 512 * kind;
  for (int s = threadIdx.x; s < 256; s += blockDim.x) fr[s] = (uint32_t)tab[2 * s] | ((uint32_t)tab[2 * s + 1] << 8);
  __syncthreads();
  if (threadIdx.x == 0) {
    cum[0] = 0;
    for (int s = 0; s < 256; s++) cum[s + 1] = cum[s] + fr[s];
  }
  __syncthreads();
  uint32_t* out = lut + (kind == 0 ? 0u : kLutLit + (uint32_t)(kind - 1) * kLutSeq);
  const uint32_t M = 1u << P;
  const uint32_t cap = kind == 0 ? kLutLit : kLutSeq;
  if (cum[256] != M) {     // unused (all-zero) table
    for (uint32_t u = threadIdx.x; u < cap; u += blockDim.x) out[u] = 0;
    return;
  }
  for (uint32_t u = threadIdx.x; u < cap; u += blockDim.x) {
    if (u >= M) { out[u] = 0; continue; }
    uint32_t lo = 0, hi = 256;   // largest s with cum[s] <= u
    while (hi - lo > 1) { uint32_t mid = (lo + hi) >> 1; if (cum[mid] <= u) lo = mid; else hi = mid; }
    const uint32_t f = fr[lo];
    out[u] = lo | ((f & 0xFFFu) << 8) | ((u - cum[lo]) << 20);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Start of a decode pass: new completion epoch, ticket reset.
__global__ void k_begin(uint32_t* ctl) {
  ctl[kCtlEpoch] += 1;
  ctl[kCtlTicket] = 0;
}

}  // namespace

// ---- host launchers (called from runtime.cpp) -------------------------------

size_t lz_decode_smem_bytes() { return sizeof(Smem); }

static DevArgs make_args(const lz_handle* h) {
  DevArgs A{};
  const ArchiveView& v = h->av;
  A.arc = v.base;
  A.n = v.n;
  A.off_dir = v.off_dir;
  A.off_dep_ptr = v.off_dep_ptr;
  A.off_dep_idx = v.off_dep_idx;
  A.off_payload = v.off_payload;
  A.bl = v.block_log2;
  A.w = v.offset_width;
  A.m = v.min_match;
  A.lit_lanes = v.lit_lanes;
  A.seq_lanes = v.seq_lanes;
  for (int k = 0; k < 4; k++) A.P[k] = v.prob_bits[k];
  A.lut = h->ws.lut;
  A.flags = h->ws.flags;
  A.ctl = h->ws.ctl;
  A.spin_limit = h->tune.spin_limit ? h->tune.spin_limit : (1u << 20);
  return A;
}

static int launch_ok(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lz_fail(LZ_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return LZ_OK;
}

int lz_launch_setup(lz_handle* h, hipStream_t s) {
  const ArchiveView& v = h->av;
  hipLaunchKernelGGL(k_build_lut, dim3(4), dim3(256), 0, s, v.base, v.off_tables, v.prob_bits[0],
                     v.prob_bits[1], v.prob_bits[2], v.prob_bits[3], h->ws.lut);
  const uint64_t nb = v.n_blocks;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(4096, (nb + 255) / 256 + 1);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, h->ws.flags, nb, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, h->ws.mark, nb, 0u);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, h->ws.addr, nb, 0ull);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, h->ws.ctl, (uint64_t)kCtlWords, 0u);
  return launch_ok("lz_open setup kernels");
}

int lz_launch_decode_all(lz_handle* h, uint8_t* out, hipStream_t s) {
  DevArgs A = make_args(h);
  A.queue = h->ws.queue;
  A.out = out;
  const size_t smem = sizeof(Smem);
  const uint32_t slots = (uint32_t)(h->n_cu * std::max(1u, h->tune.wg_per_cu));
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, h->ws.ctl);
  if (h->tune.sync_mode == 1) {
    A.persistent = 1;
    A.q_begin = 0;
    A.q_end = (uint32_t)h->av.n_blocks;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(slots, std::max<uint64_t>(1, h->av.n_blocks));
    hipLaunchKernelGGL(k_decode, dim3(grid), dim3(kWG), smem, s, A);
  } else {
    uint32_t base = 0;
    for (uint32_t L = 0; L < h->av.n_levels; L++) {
      const uint32_t c = h->level_count[L];
      if (c) {
        A.q_begin = base;
        A.q_end = base + c;
        hipLaunchKernelGGL(k_decode, dim3(std::min(c, slots)), dim3(kWG), smem, s, A);
      }
      base += c;
    }
  }
  return launch_ok("lz_decode_all");
}

// ---- verification: per-block FNV-1a-64 against the directory -----------------
namespace {

__global__ void k_fnv_blocks(const uint8_t* arc, uint64_t off_dir, const uint8_t* out, uint64_t n,
                             uint32_t bl, uint64_t nb, uint64_t* hashes, uint32_t* ctl) {
  const uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const uint64_t sb = b << bl, B = 1ull << bl;
  const uint64_t len = sb + B <= n ? B : n - sb;
  uint64_t h = kFnvBasis;
  const uint4* p = reinterpret_cast<const uint4*>(out + sb);
  uint64_t i = 0;
  for (; i + 16 <= len; i += 16) {
    const uint4 v = p[i >> 4];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int k = 0; k < 4; k++) h = (h ^ ((w[q] >> (8 * k)) & 0xFFu)) * kFnvPrime;
  }
  for (; i < len; i++) h = (h ^ out[sb + i]) * kFnvPrime;
  hashes[b] = h;
  if (h != ld64(arc + off_dir + b * kDirEntry + 24)) latch(ctl, kStHash);
}

__global__ void k_fnv_tree(const uint64_t* hashes, uint64_t nb, uint64_t* tree) {
  uint64_t h = kFnvBasis;
  for (uint64_t b = 0; b < nb; b++) {
    const uint64_t v = hashes[b];
    for (int k = 0; k < 8; k++) h = (h ^ ((v >> (8 * k)) & 0xFFu)) * kFnvPrime;
  }
  *tree = h;
}

}  // namespace

int lz_launch_verify(lz_handle* h, const uint8_t* d_out, uint64_t* d_tree, void* scratch, hipStream_t s) {
  const uint64_t nb = h->av.n_blocks;
  uint64_t* hashes = reinterpret_cast<uint64_t*>(scratch);
  if (nb) {
    if ((uintptr_t)d_out & 15) return lz_fail(LZ_EINVAL, "lz_verify: output must be 16-byte aligned");
    hipLaunchKernelGGL(k_fnv_blocks, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, s, h->av.base,
                       h->av.off_dir, d_out, h->av.n, h->av.block_log2, nb, hashes, h->ws.ctl);
  }
  hipLaunchKernelGGL(k_fnv_tree, dim3(1), dim3(1), 0, s, hashes, nb, d_tree);
  return launch_ok("lz_verify");
}

int lz_launch_requests(lz_handle*, const lz_request*, const uint32_t*, uint64_t, uint64_t, uint64_t,
                       const int64_t*, uint8_t*, uint64_t, uint64_t*, void*, uint64_t, hipStream_t) {
  return lz_fail(LZ_EINVAL, "request decoding is not built yet");
}
