// Device decoder for container format v2 on gfx950 (CDNA4, wave64).
//
// One workgroup of 256 threads (4 waves) decodes one 16 KiB block at a time
// into an LDS tile:
//   0. the block's payload prefix is copied into LDS and the four stream
//      headers are parsed from that copy;
//   1. three waves decode the command (CMD), match-length (MLEN) and offset
//      (OFF) streams, one each, reading their rANS words from the LDS copy;
//   2. one block-wide scan turns literal-run and match lengths into literal
//      and output positions (command placement), counts the matches whose
//      source touches the block itself in sequence order, and lists the
//      matches whose source lies wholly in earlier blocks;
//   3. the literal stream's 64-lane groups are decoded by one wave each, every
//      literal written straight to its output position in the tile; then the
//      matches from earlier blocks are copied from HBM;
//   4. the matches whose source touches the block are resolved in dependency
//      passes by wave 0: a match is copied once every earlier match that
//      writes into its source window is done; byte-sequential overlap is
//      unrolled by period.  Meanwhile waves 1..3 do stages 0 and 1 of the
//      workgroup's next block (its payload prefix goes into the literal
//      rings, idle until the next literal stage);
//   5. the tile is written to HBM with 16-byte stores.
// Blocks are taken in dependency-level order ("wavefront" order, paper:
// Background section): either one launch per level, or one cooperative
// launch whose workgroups walk the levels with a grid barrier between them.
// No MFMA: nothing here is a contraction.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lz_internal.h"

namespace {

constexpr uint32_t kWG = 256;
constexpr uint32_t kWaves = kWG / 64;
constexpr uint32_t kB = 1u << kMaxBlockLog2;      // largest block: 16 KiB tile
constexpr uint32_t kMaxSeq = 1025;                // B/m + 1 for B = 16 KiB, m = 16
constexpr uint32_t kLutLit = 1u << kMaxPLit;      // 4096 packed literal entries
constexpr uint32_t kL = 1u << 16;                 // rANS state lower bound
constexpr uint32_t kFastLen = 64;                 // in-block matches copied by one lane
constexpr uint32_t kClkSlots = 16;                // stage clocks: 9 stages, block count, events
constexpr uint32_t kPrepRing = kWaves * 256 * 6;  // bytes of the two literal rings

// Stage clocks (instrumented build only, -DLZ_STAGE_CLOCKS): a barrier, then
// thread 0 adds the cycles since the previous mark to stage i.  The product
// build compiles these to nothing.
#ifdef LZ_STAGE_CLOCKS
#define CLK_START(S) do { if (threadIdx.x == 0) (S).clk_last = __builtin_readcyclecounter(); } while (0)
#define CLK_MARK(S, i)                                          \
  do {                                                          \
    __syncthreads();                                            \
    if (threadIdx.x == 0) {                                     \
      const uint64_t c_ = __builtin_readcyclecounter();         \
      (S).clk[i] += c_ - (S).clk_last;                          \
      (S).clk_last = c_;                                        \
    }                                                           \
  } while (0)
// event counters (slots 10..15): CLK_ADD(S, i, v) by lane 0 of wave 0
#define CLK_ADD(S, i, v) do { if (threadIdx.x == 0) (S).clk[i] += (v); } while (0)
// the same for lane 0 of wave 1
#define CLK_ADD1(S, i, v) do { if (threadIdx.x == 64) (S).clk[i] += (v); } while (0)
#define CLK_NOW() __builtin_readcyclecounter()
#else
#define CLK_START(S) do { } while (0)
#define CLK_MARK(S, i) do { } while (0)
#define CLK_ADD(S, i, v) do { } while (0)
#define CLK_ADD1(S, i, v) do { } while (0)
#define CLK_NOW() 0ull
#endif

// All LDS is static (52,832 B: three workgroups per CU).
struct Smem {
  uint32_t lut[kLutLit];       // literal decode entries: symbol | f << 8 | (slot - c) << 20
  alignas(16) uint8_t tile[kB];// output tile; until stage 3 a copy of the payload prefix
  uint16_t cum[3][257];        // CMD, MLEN, OFF cumulative frequencies
  uint8_t bkt[3][256];         // per stream: symbol owning the first slot of each bucket
  uint16_t lit[kMaxSeq + 1];   // LL, then literal start of each sequence ([ns] = n_lit);
                               // stage 4: destination of in-block match a
  uint16_t out[kMaxSeq + 1];   // ML, then output start of each sequence ([ns] = block length);
                               // stage 4: length of in-block match a
  uint32_t oflo[kMaxSeq];      // absolute source offsets, low 32 bits; stage 4: packed
                               // source, period and dependency flag of in-block match a
  uint8_t ofhi[kMaxSeq + 3];   // offset bits 32..39
  uint16_t lst[kMaxSeq];       // [0, n_ext): matches from earlier blocks (any order);
                               // [kMaxSeq - n_in, kMaxSeq): in-block matches, last first;
                               // stage 4: dependency range of in-block match a
  union {
    struct {
      uint16_t ring[kWaves][256];  // rANS words of the literal stream staged per wave
      uint32_t ringe[kWaves][256]; // table entry of each staged word's slot
    };
    alignas(16) uint8_t prep[kPrepRing];   // between literal stages: the next block's
                                           // payload prefix (prep_ring)
  };
  uint16_t fdst[64], flen[64], frng[64];   // at most 64 in-block matches: destination,
  uint32_t fpk[64];                        // length, dependency range, source | period
  uint32_t pst[7];             // literal record of the prepared block
  uint32_t pdir[4];            // its payload offset (low, high word), sequences, literals
  uint32_t plw[kWaves], pln[kWaves];   // its literal groups' first words and word counts
  uint32_t pok;                // prepared block: records valid
  uint32_t dummy[64];          // target of the masked-off lanes' byte stores
  uint32_t scan[3][kWaves];
  uint32_t perr[3];            // prepared block: short stream k failed its checks
  uint32_t item, err, next, nin;
#ifdef LZ_STAGE_CLOCKS
  uint64_t clk[kClkSlots], clk_last;
#endif
};

struct DevArgs {
  const uint8_t* arc;
  uint64_t n, off_tables, off_dir, off_dep_ptr, off_dep_idx, off_payload;
  uint32_t bl, w, m, lit_lanes, seq_lanes;
  uint32_t P[4];
  const uint32_t* lut;      // workspace literal LUT image
  const uint32_t* queue;    // block ids in level order
  const uint32_t* qptr;     // request mode: device slice bounds (q_begin/q_end index it)
  uint32_t q_begin, q_end;  // static slice of the queue
  uint8_t* out;             // whole-file output base (direct mode)
  const uint64_t* addr;     // request mode: per-block device address, or null
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
// 16 bytes per lane straight from global memory into LDS, without registers
// (global_load_lds_dwordx4): lane k's bytes land at dst + 16 k, dst being the
// wave's uniform LDS address.  The compiler does not track the LDS write:
// lds_dma_wait() (vmcnt(0)) must come before any read of the bytes.
__device__ __forceinline__ void lds_dma16(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma_wait() {
  __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0), expcnt and lgkmcnt untouched
}
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void latch(uint32_t* ctl, uint32_t bits) {
  __hip_atomic_fetch_or(ctl + kCtlStatus, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Watchdog: latch the status bit and, for the first one, what was waited on
// (site 1 = decode dependency flag, 2 = closure entry, 3 = closure end).
__device__ __forceinline__ void watchdog(uint32_t* ctl, uint32_t site, uint32_t a, uint32_t b,
                                         uint32_t seen, uint32_t want) {
  if (__hip_atomic_fetch_or(ctl + kCtlStatus, kStWatchdog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStWatchdog) return;
  ctl[kCtlDiag + 0] = site;
  ctl[kCtlDiag + 1] = a;
  ctl[kCtlDiag + 2] = b;
  ctl[kCtlDiag + 3] = seen;
  ctl[kCtlDiag + 4] = want;
}

// True once any wait of the current call has timed out: every later wait
// gives up at once, so a call that cannot finish ends after one time-out.
__device__ __forceinline__ bool watchdog_fired(const uint32_t* ctl) {
  return __hip_atomic_load(const_cast<uint32_t*>(ctl) + kCtlStatus, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kStWatchdog;
}

// One stream record header (wave-uniform fields).
struct Stream {
  uint32_t mode, csym, K, n, nw, blen, body;
};

// Parse and check the record at *off (16-byte aligned) of the LDS copy `hp` of
// the first hlen payload bytes; records end within plen.  With `staged` the
// whole record must lie in the copy (the short streams are decoded from it).
__device__ __forceinline__ bool parse_stream(const uint8_t* hp, uint32_t hlen, uint32_t plen,
                                             uint32_t* off, uint32_t want, uint32_t maxK,
                                             bool staged, Stream& s) {
  if (*off + 16 > hlen) return false;
  const uint4 h = *reinterpret_cast<const uint4*>(hp + *off);
  s.mode = uni(h.x & 0xFFu);
  s.csym = uni((h.x >> 8) & 0xFFu);
  s.K = uni(h.x >> 16);
  s.n = uni(h.y);
  s.nw = uni(h.z);
  s.blen = uni(h.w);
  s.body = *off + 16;
  if (s.n != want) return false;
  if (staged && (uint64_t)s.body + s.blen > hlen) return false;
  switch (s.mode) {
    case kModeEmpty: if (s.n || s.blen) return false; break;
    case kModeConst: if (!s.n || s.blen) return false; break;
    case kModeRaw: if (s.blen != s.n || s.body + s.blen > plen) return false; break;
    case kModeRans: {
      const uint32_t G = (s.K + 63) >> 6;
      if (s.K < 1 || s.K > maxK || !s.n || s.body + s.blen > plen) return false;
      if ((uint64_t)s.blen != 4ull * s.K + 4ull * G + 2ull * s.nw) return false;
      if ((uint64_t)s.body + 4ull * s.K + 4ull * G > hlen) return false;
      const uint32_t* cnt = reinterpret_cast<const uint32_t*>(hp + s.body + 4 * s.K);
      uint64_t sum = 0;
      for (uint32_t g = 0; g < G; g++) sum += uni(cnt[g]);
      if (sum != s.nw) return false;
      break;
    }
    default: return false;
  }
  *off = s.body + ((s.blen + 15u) & ~15u);
  return true;
}

// Symbol owning slot u of a short stream, packed like a literal LUT entry.
// The bucket of u (2^bs slots) names the owner of its first slot; the owner
// of u is that symbol or one of the at most 2^bs - 1 symbols after it.
__device__ __forceinline__ uint32_t bucket_sym(const uint16_t* cum, const uint8_t* bkt,
                                               uint32_t bs, uint32_t u) {
  uint32_t s = bkt[u >> bs];
  uint32_t c0 = cum[s], c1 = cum[s + 1];
  while (c1 <= u && s < 255) {
    s++;
    c0 = c1;
    c1 = cum[s + 1];
  }
  return s | (((c1 - c0) & 0xFFFu) << 8) | ((u - c0) << 20);
}

// Decode a short rANS stream (one group of K <= 64 lanes) with one wave.  The
// record lies in the LDS copy `body`, so words are read from there directly.
// Lane k decodes the run of consecutive symbols starting at k*R + min(k, e),
// R = n / K, e = n mod K (container lane layout); round r decodes symbol r of
// every run still going, renormalisation words are taken in ascending lane
// order within a round.  `put.start(i)` positions lane state at symbol i and
// `put(v)` stores the lane's next symbol.  True if every state ends at 2^16 and
// every word of the group was read.
template <class Put>
__device__ bool short_rans(const uint8_t* body, const Stream& s, uint32_t P, const uint16_t* cum,
                           const uint8_t* bkt, uint32_t bs, Put& put) {
  const uint32_t lane = lane_id();
  const uint32_t K = s.K, n = s.n;
  const bool lane_ok = lane < K;
  const uint32_t nwg = uni(*reinterpret_cast<const uint32_t*>(body + 4 * K));
  const uint16_t* W = reinterpret_cast<const uint16_t*>(body + 4 * K + 4);
  const uint32_t lastw = nwg ? nwg - 1 : 0;
  uint32_t x = lane_ok ? *reinterpret_cast<const uint32_t*>(body + 4 * lane) : kL;
  bool ok = x >= kL && nwg == s.nw;
  const uint32_t R = n / K, e = n - R * K;
  put.start(lane * R + min(lane, e));
  const uint32_t mask = (1u << P) - 1;
  uint32_t pos = 0;
  auto round = [&](bool act) {
    if (act) {
      const uint32_t en = bucket_sym(cum, bkt, bs, x & mask);
      x = __umul24((en >> 8) & 0xFFFu, x >> P) + (en >> 20);
      put(en & 0xFFu);
    }
    const bool need = act && x < kL;
    const uint64_t bal = __ballot(need);
    if (need) x = (x << 16) | (uint32_t)W[min(pos + mbcnt(bal), lastw)];
    pos += (uint32_t)__popcll(bal);
  };
  for (uint32_t r = 0; r < R; r++) round(lane_ok);
  if (e) round(lane_ok && lane < e);
  ok = ok && (!lane_ok || x == kL) && pos == nwg;
  return __ballot(!ok) == 0;
}

// The first kPreSlices 128-word slices of a literal group, its lanes' initial
// states and its word range, loaded right after the stream headers are parsed
// so that their HBM latency is spent on stages 1 and 2.  Word loads are
// clamped into the group (a group without words reads the first state
// instead), so every load stays inside the record; a corrupt stream that
// consumes more words than the group holds fails pos == nwg.
constexpr uint32_t kPreSlices = 3;
struct LitPre {
  uint32_t w[2 * kPreSlices];   // w[2 s + h] = word 128 s + 64 h + lane
  uint32_t x, woff, nwg;
};

__device__ __forceinline__ const uint16_t* lit_words(const uint8_t* body, uint32_t K, const LitPre& L) {
  const uint32_t G = (K + 63) >> 6;
  return L.nwg ? reinterpret_cast<const uint16_t*>(body + 4 * K + 4 * G) + L.woff
               : reinterpret_cast<const uint16_t*>(body);
}

// body: the record body in HBM; woff, nwg: the group's first word and word
// count (prefix sums of the group word counts, done when the block was
// prepared)
__device__ __forceinline__ void lit_prefetch(const uint8_t* body, uint32_t K, uint32_t g,
                                             uint32_t woff, uint32_t nwg, LitPre& L) {
  const uint32_t lane = lane_id(), k = (g << 6) + lane;
  L.woff = woff;
  L.nwg = nwg;
  const uint16_t* W = lit_words(body, K, L);
  const uint32_t lastw = L.nwg ? L.nwg - 1 : 0;
#pragma unroll
  for (uint32_t i = 0; i < 2 * kPreSlices; i++) L.w[i] = (uint32_t)W[min(64 * i + lane, lastw)];
  L.x = k < K ? ld32(body + 4 * k) : kL;
}

// Literal stream, one 64-lane group g of K lanes, every lane active for R
// rounds (a full group) or under `act` masks (FULL false).  Same symbols,
// words and checks as short_rans; the group's 16-bit words are staged from HBM
// through the wave's LDS ring (two 128-word slices, the next two slices in
// registers), and every staged word carries the table entry of the slot it
// starts (after x = (x << 16) | w the next slot is w mod 2^P), so a round
// makes one LDS round trip: renormalising lanes read word and entry, the
// others look up their new slot.  Each symbol goes straight to its tile
// position tp; when tp reaches the end of the lane's current literal run
// (tpend) the lane moves to the next sequence that has literals.
template <uint32_t P, bool FULL>
__device__ bool lit_group(const uint8_t* body, uint32_t K, uint32_t n, uint32_t nw_total, uint32_t g,
                          Smem& S, uint32_t wv, uint32_t ns, const LitPre& L) {
  const uint32_t lane = lane_id();
  const uint32_t k = (g << 6) + lane;
  const bool lane_ok = k < K;
  const uint32_t nwg = L.nwg;
  const uint16_t* W = lit_words(body, K, L);
  const uint32_t lastw = nwg ? nwg - 1 : 0;
  auto ldw = [&](uint32_t idx) -> uint32_t { return (uint32_t)W[min(idx, lastw)]; };
  constexpr uint32_t mask = (1u << P) - 1;
  uint16_t* ring = S.ring[wv];
  uint32_t* ringe = S.ringe[wv];
  uint32_t x = L.x;
  bool ok = x >= kL && L.woff + nwg <= nw_total;
  // slices 0 and 1 into the ring, slices 2..5 wait in registers
  {
    uint32_t en[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) en[q] = S.lut[L.w[q] & mask];
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
      ring[64 * q + lane] = (uint16_t)L.w[q];
      ringe[64 * q + lane] = en[q];
    }
  }
  // slice 2 waits in registers (u0, u1); staging it loads the next slice
  // straight into the same registers, so no register moves follow the loads
  // and their wait falls one slice later
  static_assert(kPreSlices == 3, "the ring holds slices 0 and 1, registers slice 2");
  uint32_t u0 = L.w[4], u1 = L.w[5];
  uint32_t e = S.lut[x & mask];
  uint32_t pos = 0;
  const uint32_t R = n / K, ex = n - R * K;
  // the lane's first literal i0 lies in sequence j: lit[j] <= i0 < lit[j+1]
  const uint32_t i0 = min(k * R + min(k, ex), n ? n - 1 : 0);
  uint32_t j = 0;
  {
    uint32_t lo = 0, hi = ns - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (S.lit[mid] <= i0) lo = mid; else hi = mid - 1;
    }
    j = lo;
  }
  uint32_t tp = i0 - S.lit[j] + S.out[j];
  uint32_t tpend = S.out[j] + (uint32_t)S.lit[j + 1] - S.lit[j];
  // literal runs of the next three sequences in registers (start, end in the
  // tile), so that moving to the next run reads no LDS; jq = last queued one
  uint32_t q1, e1, q2, e2, q3, e3, jq = min(j + 3, ns - 1);
  {
    const uint32_t j1 = min(j + 1, ns - 1), j2 = min(j + 2, ns - 1), j3 = jq;
    q1 = S.out[j1]; e1 = q1 + (uint32_t)S.lit[j1 + 1] - S.lit[j1];
    q2 = S.out[j2]; e2 = q2 + (uint32_t)S.lit[j2 + 1] - S.lit[j2];
    q3 = S.out[j3]; e3 = q3 + (uint32_t)S.lit[j3 + 1] - S.lit[j3];
  }
  auto round = [&](bool act) {
    if (act) {
      S.tile[tp] = (uint8_t)e;
      x = __umul24((e >> 8) & 0xFFFu, x >> P) + (e >> 20);
      tp++;
    }
    const bool need = act && x < kL;
    const uint64_t bal = __ballot(need);
    const uint32_t q = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, pos)) & 255u;
    const uint32_t w = ring[q];
    e = need ? ringe[q] : S.lut[x & mask];
    x = need ? (x << 16) | w : x;
    pos += (uint32_t)__popcll(bal);
    // end of the lane's literal run in this sequence: the next sequence
    // with literals (every literal index below n_lit has one), from the
    // register queue while it lasts, else from the tables
    if (act && tp == tpend) {
      for (uint32_t hop = 0; hop < 3 && tp == tpend; hop++) {
        tp = q1; tpend = e1;
        q1 = q2; e1 = e2;
        q2 = q3; e2 = e3;
        q3 = e3;                          // empty run: exhausts the queue
      }
      if (tp == tpend) {
        uint32_t nj = jq + 1;
        while (nj + 1 < ns && S.lit[nj + 1] == S.lit[nj]) nj++;
        jq = min(nj, ns - 1);
        tp = S.out[jq];
        tpend = tp + (uint32_t)S.lit[jq + 1] - S.lit[jq];
        q1 = q2 = q3 = e1 = e2 = e3 = tpend;
      }
    }
  };
  // A round that enters slice s0+1 stages slice s0+2 from the registers into
  // the ring half of slice s0 and loads slice s0+kPreSlices into them. Written
  // out in this scope: inside the round helper, which takes its state by
  // reference, the registers would be spilled to a private array.
#define LZ_ROUND(act)                                                   \
  {                                                                     \
    const uint32_t s0 = pos >> 7;                                       \
    round(act);                                                         \
    if ((pos >> 7) != s0) {                                             \
      __builtin_amdgcn_wave_barrier(); /* every lane read slice s0 */   \
      const uint32_t d = ((s0 & 1) << 7) + lane;                        \
      const uint32_t b3 = (s0 + kPreSlices) << 7;                       \
      const uint32_t ea = S.lut[u0 & mask], eb = S.lut[u1 & mask];      \
      ring[d] = (uint16_t)u0;                                           \
      ring[d + 64] = (uint16_t)u1;                                      \
      ringe[d] = ea;                                                    \
      ringe[d + 64] = eb;                                               \
      if (b3 < nwg) {                  /* words left to fetch */        \
        u0 = ldw(b3 + lane);                                            \
        u1 = ldw(b3 + 64 + lane);                                       \
      }                                                                 \
    }                                                                   \
  }
  if (FULL) {
    for (uint32_t r = 0; r < R; r++) LZ_ROUND(true)
  } else {
    for (uint32_t r = 0; r < R; r++) LZ_ROUND(lane_ok)
  }
  if (ex) round(lane_ok && k < ex);     // no read follows: nothing to stage
#undef LZ_ROUND
  ok = ok && (!lane_ok || x == kL) && pos == nwg;
  return __ballot(!ok) == 0;
}

template <uint32_t P>
__device__ bool lit_group_p(const uint8_t* body, uint32_t K, uint32_t n, uint32_t nw, uint32_t g,
                            Smem& S, uint32_t wv, uint32_t ns, const LitPre& L) {
  if ((g << 6) + 64 <= K) return lit_group<P, true>(body, K, n, nw, g, S, wv, ns, L);
  return lit_group<P, false>(body, K, n, nw, g, S, wv, ns, L);
}

// Source byte at absolute position a (an earlier block): direct mode reads the
// whole-file output; request mode goes through the per-block address table.
__device__ __forceinline__ uint32_t src_byte(const DevArgs& A, uint64_t a, bool& bad) {
  if (!A.addr) return A.out[a];
  const uint64_t base = A.addr[a >> A.bl];
  if (!base) { bad = true; return 0; }
  return reinterpret_cast<const uint8_t*>(base)[a & ((1ull << A.bl) - 1)];
}

// Inclusive scan over the 64 lanes of a wave with DPP moves (no LDS): shifts
// by 1, 2, 4 and 8 inside each 16-lane row, then the last lane of row 0 is
// added to row 1 and of row 2 to row 3 (row_bcast:15), then lane 31 to rows
// 2 and 3 (row_bcast:31).  Lanes whose DPP source is outside the row read 0.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}

// Block-wide exclusive scans of three counts at once; tot[] receives the sums.
__device__ void block_scan3(Smem& S, const uint32_t v[3], uint32_t pre[3], uint32_t tot[3]) {
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  uint32_t incl[3];
#pragma unroll
  for (int f = 0; f < 3; f++) {
    incl[f] = wave_scan(v[f]);
    if (lane == 63) S.scan[f][wv] = incl[f];
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 3; f++) {
    uint32_t base = 0, all = 0;
#pragma unroll
    for (uint32_t q = 0; q < kWaves; q++) {
      const uint32_t w = S.scan[f][q];
      if (q < wv) base += w;
      all += w;
    }
    pre[f] = base + incl[f] - v[f];
    tot[f] = all;
  }
  // no closing barrier: S.scan is next written by the next block's scan,
  // many barriers later
}

// Small-stream symbol lookup: binary search of slot u in a 257-entry
// cumulative table.
__device__ __forceinline__ uint32_t search_sym(const uint16_t* cum, uint32_t u) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = 128; step; step >>= 1)
    if (cum[lo + step] <= u) lo += step;
  return lo;
}

// Writes the decoded values of a short stream: symbol i is byte plane i / ns
// of value i mod ns (values stored byte-plane major); a lane's symbols are
// consecutive, so its (plane, index) pair advances by one each call.
struct PutPlanes {
  uint8_t* lo;      // planes 0..lo_planes-1: byte `plane` of the value at lo + stride * idx
  uint8_t* hi;      // plane 4 (offsets only): hi[idx]
  uint32_t stride, ns, idx, plane;
  __device__ void start(uint32_t i) {
    plane = i / ns;
    idx = i - plane * ns;
  }
  __device__ void operator()(uint32_t v) {
    if (plane < 4) lo[stride * idx + min(plane, stride - 1)] = (uint8_t)v;
    else hi[idx] = (uint8_t)v;
    if (++idx == ns) { idx = 0; plane++; }
  }
};

// Where block b's payload lies and how many sequences and literals it holds.
struct BlockDir {
  uint64_t poff;
  uint32_t plen, ns, nlit, blen;
};

__device__ __forceinline__ BlockDir block_dir(const DevArgs& A, uint32_t b) {
  const uint64_t B = 1ull << A.bl, sb = (uint64_t)b << A.bl;
  const uint8_t* de = A.arc + A.off_dir + (uint64_t)b * kDirEntry;
  BlockDir d;
  d.poff = ld64(de);
  d.plen = ld32(de + 8);
  d.ns = ld32(de + 12);
  d.nlit = ld32(de + 16);
  d.blen = (uint32_t)((sb + B <= A.n) ? B : A.n - sb);
  return d;
}

// The four stream records (CMD, MLEN, OFF, LIT) parsed and checked from the
// LDS copy hp of the block's first hlen payload bytes (every thread parses
// the same bytes, so the result is wave-uniform).
__device__ __forceinline__ bool parse_records(const DevArgs& A, const BlockDir& d, const uint8_t* hp,
                                              uint32_t hlen, Stream& sc, Stream& sm, Stream& so,
                                              Stream& sl) {
  uint32_t off = 0;
  bool ok = d.ns >= 1 && d.ns <= kMaxSeq && d.nlit <= d.blen && (d.poff & 15) == 0;
  ok = ok && parse_stream(hp, hlen, d.plen, &off, 2 * d.ns, A.seq_lanes, true, sc);
  ok = ok && parse_stream(hp, hlen, d.plen, &off, 2 * d.ns, A.seq_lanes, true, sm);
  ok = ok && parse_stream(hp, hlen, d.plen, &off, A.w * d.ns, A.seq_lanes, true, so);
  ok = ok && parse_stream(hp, hlen, d.plen, &off, d.nlit, A.lit_lanes, false, sl);
  return ok;
}

// Short stream `role` of a block with ns sequences, by one wave: 0 CMD ->
// lit[] (LL), 1 MLEN -> out[] (ML), 2 OFF -> oflo/ofhi (absolute offsets).
__device__ bool short_stream(Smem& S, const DevArgs& A, uint32_t role, const Stream& s,
                             const uint8_t* hp, uint32_t ns) {
  const uint32_t lane = lane_id();
  PutPlanes put;
  put.ns = ns;
  if (role < 2) {
    put.lo = role == 0 ? reinterpret_cast<uint8_t*>(S.lit) : reinterpret_cast<uint8_t*>(S.out);
    put.hi = put.lo;
    put.stride = 2;
  } else {
    put.lo = reinterpret_cast<uint8_t*>(S.oflo);
    put.hi = S.ofhi;
    put.stride = 4;
    // offsets narrower than 5 bytes: clear the planes the stream does not hold
    for (uint32_t j = lane; j < ns; j += 64) { S.oflo[j] = 0; S.ofhi[j] = 0; }
    __builtin_amdgcn_wave_barrier();
  }
  if (s.mode == kModeRans) {
    const uint32_t P = A.P[1 + role];
    const uint32_t bs = P > 8 ? P - 8 : 0u;
    return short_rans(hp + s.body, s, P, S.cum[role], S.bkt[role], bs, put);
  }
  if (s.mode == kModeRaw || s.mode == kModeConst) {
    const uint8_t* src = hp + s.body;
    for (uint32_t i = lane; i < s.n; i += 64) {
      put.start(i);
      put(s.mode == kModeRaw ? (uint32_t)src[i] : s.csym);
    }
  }
  return true;
}

// What the later stages need of the prepared block (one thread): its
// directory fields, the literal record and the literal groups' word ranges
// (the group word counts lie in the copy hp: parse_stream checks that).
__device__ __forceinline__ void put_prep(Smem& S, const BlockDir& d, const Stream& s, const uint8_t* hp,
                                         bool ok) {
  S.pdir[0] = (uint32_t)d.poff; S.pdir[1] = (uint32_t)(d.poff >> 32); S.pdir[2] = d.ns; S.pdir[3] = d.nlit;
  S.pst[0] = s.mode; S.pst[1] = s.csym; S.pst[2] = s.K; S.pst[3] = s.n;
  S.pst[4] = s.nw; S.pst[5] = s.blen; S.pst[6] = s.body;
  const uint32_t G = ok && s.mode == kModeRans ? (s.K + 63) >> 6 : 0u;
  const uint32_t* cnt = reinterpret_cast<const uint32_t*>(hp + s.body + 4 * s.K);
  uint32_t w = 0;
  for (uint32_t g = 0; g < kWaves; g++) {
    const uint32_t c = g < G ? cnt[g] : 0u;
    S.plw[g] = w;
    S.pln[g] = c;
    w += c;
  }
}

// Stages 0 and 1 of block b ("preparing" it): the payload prefix is copied
// into LDS, the four stream records are parsed and checked, and the CMD, MLEN
// and OFF streams are decoded into the sequence tables.  The literal record
// goes to S.pst with the directory fields and literal group word ranges
// (put_prep), the outcome to S.pok; a short stream that fails its checks sets
// S.perr[k] (written by the wave that decoded stream k, 0 or 1).
//
// prep_tile: all four waves.  The first min(plen, 16 KiB) payload bytes go
// into the tile (free until the literal stage) with one round of 16-byte
// loads; waves 0..2 decode the short streams from there (at most about 9.3 KB
// with their headers for 1025 sequences).  Corrupt records are latched.
__device__ __forceinline__ void prep_tile(Smem& S, const DevArgs& A, uint32_t b) {
  const uint32_t t = threadIdx.x, wv = uni(t >> 6), lane = lane_id();
  const BlockDir d = block_dir(A, b);
  const uint8_t* pay = A.arc + A.off_payload + d.poff;
  CLK_START(S);
  const uint32_t hlen = min(d.plen, kB);
  {
    const uint32_t n16 = hlen >> 4;
    const bool tail = t < (hlen & 15u);              // bytes past the last 16
    const uint32_t tb = tail ? (uint32_t)pay[(hlen & ~15u) + t] : 0u;
    if (((uintptr_t)pay & 15u) == 0) {   // straight into LDS, one HBM round trip
#pragma unroll 1
      for (uint32_t i = 0; i < kB / (16 * kWG); i++)
        if (t + kWG * i < n16) lds_dma16(pay + 16 * (t + kWG * i), S.tile + 16 * (64 * wv + kWG * i));
      lds_dma_wait();
    } else {
      const uint4* src4 = reinterpret_cast<const uint4*>(pay);
      uint4* dst4 = reinterpret_cast<uint4*>(S.tile);
      for (uint32_t c = t; c < n16; c += kWG) dst4[c] = src4[c];
    }
    if (tail) S.tile[(hlen & ~15u) + t] = (uint8_t)tb;
  }
  if (t == 0) S.next = 0;
  __syncthreads();
  CLK_MARK(S, 0);
  Stream sc, sm, so, sl;
  const bool ok = parse_records(A, d, S.tile, hlen, sc, sm, so, sl);
  if (t == 0) {
    S.pok = ok ? 1u : 0u;
    put_prep(S, d, sl, S.tile, ok);
    if (!ok) latch(A.ctl, kStCorrupt);
  }
  CLK_MARK(S, 1);
  if (ok && wv < 3) {
    const Stream& s = wv == 0 ? sc : (wv == 1 ? sm : so);
    const bool okw = short_stream(S, A, wv, s, S.tile, d.ns);
    if (lane == 0) S.perr[wv] = okw ? 0u : 1u;
  }
  __syncthreads();
  CLK_MARK(S, 2);
}

// prep_ring: waves 1..3 only, while wave 0 resolves the previous block's
// in-block matches, so no workgroup barrier may be used.  Every wave copies
// the same first kPrepRing payload bytes into the literal rings (idle from
// the end of the literal stage to the next one) itself, so each needs only
// its own stores before it reads; waves 1..3 decode CMD, MLEN and OFF.  A
// prefix too short for the short streams and the literal record's states and
// counts (or corrupt records) leaves S.pok 0, and the block is prepared again
// by prep_tile.  The caller guarantees that the sequence tables, S.pst and
// the rings are not in use.
__device__ __forceinline__ void prep_ring(Smem& S, const DevArgs& A, uint32_t b) {
  const uint32_t wv = uni(threadIdx.x >> 6), lane = lane_id();
  const BlockDir d = block_dir(A, b);
  const uint8_t* pay = A.arc + A.off_payload + d.poff;
  const uint32_t hlen = min(d.plen, kPrepRing);
  {
    const uint32_t n16 = hlen >> 4;
    const bool tail = lane < (hlen & 15u);           // bytes past the last 16
    const uint32_t tb = tail ? (uint32_t)pay[(hlen & ~15u) + lane] : 0u;
    if (((uintptr_t)pay & 15u) == 0) {
      // every 1 KiB of the prefix at once, straight into LDS: one HBM round
      // trip (copied through registers it was one per 1 KiB, as the
      // registers are all taken here)
#pragma unroll 1
      for (uint32_t i = 0; i < kPrepRing / 1024; i++)   // not unrolled: no hoisted addresses
        if (lane + 64 * i < n16) lds_dma16(pay + 16 * (lane + 64 * i), S.prep + 1024 * i);
      lds_dma_wait();
    } else {
      const uint4* src4 = reinterpret_cast<const uint4*>(pay);
      uint4* dst4 = reinterpret_cast<uint4*>(S.prep);
      for (uint32_t c = lane; c < n16; c += 64) dst4[c] = src4[c];
    }
    if (tail) S.prep[(hlen & ~15u) + lane] = (uint8_t)tb;
  }
  __builtin_amdgcn_wave_barrier();
  Stream sc, sm, so, sl;
  const bool ok = parse_records(A, d, S.prep, hlen, sc, sm, so, sl);
  bool okw = true;
  if (ok) {
    const uint32_t role = wv - 1;
    const Stream& s = role == 0 ? sc : (role == 1 ? sm : so);
    okw = short_stream(S, A, role, s, S.prep, d.ns);
  }
  if (ok && lane == 0) S.perr[wv - 1] = okw ? 0u : 1u;
  if (wv == 1 && lane == 0) {
    S.pok = ok ? 1u : 0u;
    put_prep(S, d, sl, S.prep, ok);
    S.next = 0;
  }
}

// Decode block b, prepared by prep_tile or prep_ring (S.pok, S.pst and the
// sequence tables hold its stages 0 and 1), into the LDS tile and store it.
// nb is the workgroup's next block or ~0u; the result is true when nb has
// been prepared meanwhile, by waves 1..3 while wave 0 resolved b's in-block
// matches.  Every loop below is bounded by values read from global memory
// (directory, stream headers).
__device__ __forceinline__ bool decode_block(Smem& S, const DevArgs& A, uint32_t b, uint32_t nb) {
  const uint32_t t = threadIdx.x, wv = uni(t >> 6), lane = lane_id();
  const uint64_t B = 1ull << A.bl, sb = (uint64_t)b << A.bl;
  const uint32_t blen = (uint32_t)((sb + B <= A.n) ? B : A.n - sb);
  if (!uni(S.pok)) return false;               // corrupt records (latched by prep_tile)
  const uint64_t poff = (uint64_t)uni(S.pdir[0]) | ((uint64_t)uni(S.pdir[1]) << 32);
  const uint32_t ns = uni(S.pdir[2]), nlit = uni(S.pdir[3]);
  const uint8_t* pay = A.arc + A.off_payload + poff;
  Stream sl;
  sl.mode = uni(S.pst[0]); sl.csym = uni(S.pst[1]); sl.K = uni(S.pst[2]); sl.n = uni(S.pst[3]);
  sl.nw = uni(S.pst[4]); sl.blen = uni(S.pst[5]); sl.body = uni(S.pst[6]);
  // literal group of this wave (K <= 256: at most one per wave), fetched ahead
  const uint32_t Glit = sl.mode == kModeRans ? (sl.K + 63) >> 6 : 0u;
  LitPre lp;
  if (wv < Glit) lit_prefetch(pay + sl.body, sl.K, wv, uni(S.plw[wv]), uni(S.pln[wv]), lp);
  if (t == 0) S.err = 0;

  // ---- stage 2: command placement.  One block scan of (LL, LL + ML,
  // in-block match) counts gives literal and output positions and the order
  // of the in-block matches; the block's sequence invariants are checked.
  // Values are u16 and ns <= 1025, so no sum reaches 2^32.  A block of at
  // most 64 sequences is placed by wave 0 alone with one wave scan (no
  // workgroup barrier); waves 1..3 wait at the stage's closing barrier.
  const bool one = ns <= 64;
  if (!one || wv == 0) {
    const uint32_t per = (ns + kWG - 1) / kWG;   // <= 5
    const uint32_t j0 = min(ns, t * per), j1 = min(ns, j0 + per);
    uint32_t ll[5], ml[5];
    uint32_t v[3] = {0, 0, 0};
    bool bad = false;
#pragma unroll
    for (uint32_t q = 0; q < 5; q++) {
      const uint32_t j = j0 + q;
      ll[q] = j < j1 ? S.lit[j] : 0u;
      ml[q] = j < j1 ? S.out[j] : 0u;
      uint32_t inb = 0;
      if (j < j1 && ml[q]) {
        const uint64_t of = (uint64_t)S.oflo[j] | ((uint64_t)S.ofhi[j] << 32);
        inb = of + ml[q] > sb ? 1u : 0u;
      }
      v[0] += ll[q];
      v[1] += ll[q] + ml[q];
      v[2] += inb;
    }
    uint32_t pre[3], tot[3];
    if (one) {
#pragma unroll
      for (int f = 0; f < 3; f++) {
        const uint32_t incl = wave_scan(v[f]);
        pre[f] = incl - v[f];
        tot[f] = __builtin_amdgcn_readlane(incl, 63);
      }
    } else {
      block_scan3(S, v, pre, tot);
    }
    const uint32_t tl = tot[0], to = tot[1];
    bad |= tl != nlit || to != blen;
    uint32_t pl = pre[0], po = pre[1];
    uint32_t pin = pre[2];
#pragma unroll
    for (uint32_t q = 0; q < 5; q++) {
      const uint32_t j = j0 + q;
      if (j < j1) {
        S.lit[j] = (uint16_t)pl;
        S.out[j] = (uint16_t)po;
        const uint64_t of = (uint64_t)S.oflo[j] | ((uint64_t)S.ofhi[j] << 32);
        if (ml[q] == 0) {
          bad |= (j != ns - 1) || of != 0;
        } else {
          bad |= ml[q] < A.m || of >= sb + po + ll[q];
          if (of + ml[q] <= sb) {
            S.lst[atomicAdd(&S.next, 1u)] = (uint16_t)j;   // from earlier blocks, any order
          } else {
            S.lst[kMaxSeq - 1 - pin] = (uint16_t)j;        // in-block, in sequence order
            if (pin < 64) {                                // the common case: its fields at once
              const uint32_t d0 = po + ll[q];
              const uint64_t dabs = sb + d0;
              S.fdst[pin] = (uint16_t)d0;
              S.flen[pin] = (uint16_t)min(ml[q], blen);
              S.fpk[pin] = ((uint32_t)((int64_t)of - (int64_t)sb + 16384) & 0xFFFFu) |
                           ((dabs > of ? (uint32_t)min<uint64_t>(dabs - of, 32767) : 1u) << 16);
            }
            pin++;
          }
        }
        pl += ll[q];
        po += ll[q] + ml[q];
      }
    }
    if (t == 0) {
      S.lit[ns] = (uint16_t)min(tl, 65535u);
      S.out[ns] = (uint16_t)min(to, 65535u);
      S.nin = tot[2];
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err || S.perr[0] || S.perr[1] || S.perr[2]) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return false;
  }
  CLK_MARK(S, 3);

  // ---- stage 3: literals straight to their tile positions; external matches
  {
    bool bad = false;
    const uint32_t nx = min(S.next, ns), slot = lane >> 3, sub = lane & 7;
    // Matches with a source wholly in earlier blocks.  In whole-file mode the
    // first sixteen are started before the literal decode, four per wave (one
    // per 16-lane quarter): each lane loads two aligned source words covering
    // eight bytes of the match's first 128, so the HBM latency is spent
    // decoding; the bytes are stored after it.  The rest are copied eight per
    // wave at a time, one per 8-lane slot, each lane every eighth byte, all
    // loads in flight before the stores.
    const bool early = A.addr == nullptr;
    const uint32_t quarter = lane >> 4, qsub = lane & 15;
    uint32_t pM = 0, pd0 = 0, pw0 = 0, pw1 = 0;
    uint64_t pof = 0, pa = 0;
    if (early) {
      const uint32_t e = 4 * wv + quarter;
      const uint32_t q = e < nx ? min((uint32_t)S.lst[e], ns - 1) : 0u;
      const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
      pM = e < nx ? (uint32_t)S.out[q + 1] - S.out[q] - L : 0u;
      pof = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
      pd0 = S.out[q] + L;
      // words [pa, pa + 8) with pa = (of & ~3) + 8 * qsub cover the bytes
      // k < 128 - (of & 3) of the match; the last word may reach up to 3 bytes
      // past the match, still inside the output (the source ends at or
      // before this block's start)
      pa = (pof & ~3ull) + 8ull * qsub;
      const uint32_t* w = reinterpret_cast<const uint32_t*>(A.out + pa);
      const uint64_t lim = pof + min(pM, 128u - (uint32_t)(pof & 3));
      pw0 = pa < lim ? w[0] : 0u;
      pw1 = pa + 4 < lim ? w[1] : 0u;
    }
    if (wv < Glit) {
      const uint32_t g = wv;
      bool okg;
      switch (A.P[kLit]) {
        case 8: okg = lit_group_p<8>(pay + sl.body, sl.K, sl.n, sl.nw, g, S, wv, ns, lp); break;
        case 9: okg = lit_group_p<9>(pay + sl.body, sl.K, sl.n, sl.nw, g, S, wv, ns, lp); break;
        case 10: okg = lit_group_p<10>(pay + sl.body, sl.K, sl.n, sl.nw, g, S, wv, ns, lp); break;
        case 11: okg = lit_group_p<11>(pay + sl.body, sl.K, sl.n, sl.nw, g, S, wv, ns, lp); break;
        default: okg = lit_group_p<12>(pay + sl.body, sl.K, sl.n, sl.nw, g, S, wv, ns, lp); break;
      }
      if (!okg) bad = true;
    } else if (sl.mode == kModeRaw || sl.mode == kModeConst) {
      // one thread per literal: the sequence by binary search
      const uint8_t* src = pay + sl.body;
      for (uint32_t i = t; i < sl.n; i += kWG) {
        uint32_t lo = 0, hi = ns - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if (S.lit[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const uint32_t p = i - S.lit[lo] + S.out[lo];
        S.tile[min(p, kB - 1)] = sl.mode == kModeRaw ? src[i] : (uint8_t)sl.csym;
      }
    }
    CLK_MARK(S, 4);
    if (early) {
      const uint64_t lim = pof + min(pM, 128u - (uint32_t)(pof & 3));
#pragma unroll
      for (uint32_t u = 0; u < 8; u++) {
        const uint64_t a = pa + u;
        const uint32_t v = (u < 4 ? pw0 : pw1) >> (8 * (u & 3));
        if (a >= pof && a < lim) S.tile[pd0 + (uint32_t)(a - pof)] = (uint8_t)v;
      }
      for (uint32_t k0 = 128u - (uint32_t)(pof & 3); __ballot(k0 < pM); k0 += 128) {   // the rest
        uint32_t v[8];
        const uint8_t* p = A.out + pof + k0 + qsub;
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) v[u] = k0 + qsub + 16 * u < pM ? (uint32_t)p[16 * u] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) {
          const uint32_t k = k0 + qsub + 16 * u;
          if (k < pM && pd0 + k < blen) S.tile[pd0 + k] = (uint8_t)v[u];
        }
      }
    }
    for (uint32_t g0 = 8 * wv + (early ? 4 * kWaves : 0u); g0 < nx; g0 += 8 * kWaves) {
      const uint32_t e = g0 + slot;
      const uint32_t q = e < nx ? min((uint32_t)S.lst[e], ns - 1) : 0u;
      const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
      const uint32_t M = e < nx ? (uint32_t)S.out[q + 1] - S.out[q] - L : 0u;
      const uint64_t of = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
      const uint32_t d0 = S.out[q] + L;
      for (uint32_t k0 = 0; __ballot(k0 < M); k0 += 256) {
        uint32_t v[32];
        if (!A.addr) {                       // whole-file output: one base, byte offsets
          const uint8_t* p = A.out + of + k0 + sub;
#pragma unroll
          for (uint32_t u = 0; u < 32; u++) v[u] = k0 + sub + 8 * u < M ? (uint32_t)p[8 * u] : 0u;
        } else {
#pragma unroll
          for (uint32_t u = 0; u < 32; u++) {
            const uint32_t k = k0 + sub + 8 * u;
            v[u] = k < M ? src_byte(A, of + k, bad) : 0u;
          }
        }
#pragma unroll
        for (uint32_t u = 0; u < 32; u++) {
          const uint32_t k = k0 + sub + 8 * u;
          if (k < M && d0 + k < blen) S.tile[d0 + k] = (uint8_t)v[u];
        }
      }
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return false;
  }
  CLK_MARK(S, 5);

  // ---- stage 4: matches whose source touches the block itself.
  // With period d = p - OF, out[p+k] = out[OF + (k mod d)] for every k (the
  // byte-sequential overlap rule unrolled); only the window OF..OF+min(d,M)-1
  // is read and it is final once every earlier match writing into it is done.
  // 4a: per match a (sequence order): destination, length, block-relative
  //     source and period, and the index range of earlier in-block matches
  //     whose destinations its window meets (two binary searches over the
  //     sorted, disjoint destinations);
  // 4b: wave 0 copies them in passes over 64-entry chunks (every earlier
  //     chunk complete): a pass takes every pending match whose predecessors
  //     are done.  Short matches (at most 64 bytes, no overlap with themselves,
  //     source inside the tile) are copied by their own lane from four-byte
  //     words; the others by the whole wave, one at a time.
  // With at most 64 in-block matches (the common case) stage 2 has written
  // their fields to their own small arrays and only wave 0 works on them: the
  // sequence tables are free, and waves 1..3 prepare the next block
  // meanwhile.  With more, the fields are packed into the sequence tables and
  // 4a uses every thread.
  const uint32_t cnt = min(S.nin, ns);
  const bool small = cnt <= 64;
  uint16_t* Fd = small ? S.fdst : S.lit;     // destination
  uint16_t* Fl = small ? S.flen : S.out;     // length
  uint32_t* Fp = small ? S.fpk : S.oflo;     // source | period << 16
  uint16_t* Fr = small ? S.frng : S.lst;     // dependency range within the chunk
  uint32_t md0[5], mM[5], ms[5], md[5];
  const uint32_t per = (cnt + kWG - 1) / kWG, a0 = min(cnt, t * per), a1 = min(cnt, a0 + per);
  // dependency ranges of this thread's matches (reads Fd, Fl of earlier ones)
  auto ranges = [&]() {
#pragma unroll
    for (uint32_t u = 0; u < 5; u++) {
      const uint32_t a = a0 + u;
      if (a < a1) {
        const int32_t s = (int32_t)ms[u] - 16384;
        const uint32_t w = min(md[u], mM[u]);
        uint32_t lo = a, hi = a;
        if (s + (int32_t)w > 0) {
          const uint32_t ws = s > 0 ? (uint32_t)s : 0u, we = (uint32_t)(s + (int32_t)w);
          // lo = first earlier match whose destination ends after ws, hi =
          // first whose destination starts at or after we (hi >= lo)
          uint32_t l1 = 0, h1 = a, l2 = 0, h2 = a;
          while (l1 < h1 || l2 < h2) {
            const uint32_t m1 = (l1 + h1) >> 1, m2 = (l2 + h2) >> 1;
            const uint32_t e1 = (uint32_t)Fd[min(m1, a - 1)] + Fl[min(m1, a - 1)];
            const uint32_t b2 = Fd[min(m2, a - 1)];
            if (l1 < h1) { if (e1 > ws) h1 = m1; else l1 = m1 + 1; }
            if (l2 < h2) { if (b2 >= we) h2 = m2; else l2 = m2 + 1; }
          }
          lo = l1;
          hi = l2;
        }
        const uint32_t c0 = a & ~63u;
        const uint32_t plo = max(lo, c0) - c0, phi = max(hi, c0) - c0;   // both <= 63
        Fr[a] = (uint16_t)(plo | (phi << 8));
        Fp[a] = ms[u] | (md[u] << 16);
      }
    }
  };
  if (!small) {                              // more than 64: fields packed into the tables
#pragma unroll
    for (uint32_t u = 0; u < 5; u++) {
      const uint32_t a = a0 + u;
      const uint32_t q = a < a1 ? min((uint32_t)S.lst[kMaxSeq - 1 - a], ns - 1) : 0u;
      const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
      const uint32_t M = min((uint32_t)S.out[q + 1] - S.out[q] - L, blen);
      const uint32_t d0 = S.out[q] + L;
      const uint64_t of = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
      const uint64_t dabs = sb + d0;
      md0[u] = d0;
      mM[u] = M;
      // of + M > sb here (the source window touches the block) and of < dabs,
      // so the relative source fits in [-16384, 16384)
      ms[u] = (uint32_t)((int64_t)of - (int64_t)sb + 16384) & 0xFFFFu;
      md[u] = dabs > of ? (uint32_t)min<uint64_t>(dabs - of, 32767) : 1u;
    }
    __syncthreads();                         // Fd, Fl are the tables just read
#pragma unroll
    for (uint32_t u = 0; u < 5; u++) {
      const uint32_t a = a0 + u;
      if (a < a1) {
        Fd[a] = (uint16_t)md0[u];
        Fl[a] = (uint16_t)mM[u];
      }
    }
    __syncthreads();
    ranges();
    __syncthreads();
  }
  CLK_MARK(S, 6);
  // No workgroup barrier from here to the end of the passes: wave 0 and
  // waves 1..3 run different code.
  const bool ov = small && nb != ~0u;
  const uint64_t c4_ = CLK_NOW();
  if (wv == 0 && cnt) {
    // wave 0's passes bound this stage: it wins issue on its SIMD meanwhile
    __builtin_amdgcn_s_setprio(2);
    if (small) {                             // fields from stage 2 (before two barriers)
      if (a0 < a1) {
        const uint32_t pk = Fp[a0];
        md0[0] = Fd[a0];
        mM[0] = Fl[a0];
        ms[0] = pk & 0xFFFFu;
        md[0] = pk >> 16;
      }
      ranges();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    bool bad = false;
    // whole-wave copy of in-block match a (any length, period and source)
    auto copy_match = [&](uint32_t a) {
      const uint32_t pk = Fp[a];
      const uint32_t d0 = Fd[a], M = Fl[a];
      const int32_t s = (int32_t)(pk & 0xFFFFu) - 16384;
      const uint32_t d = (pk >> 16) & 0x7FFFu;
      // (k mod d) kept incrementally (a division only for d < 64)
      uint32_t r = d >= M ? lane : (d >= 64 ? lane : lane % d);
      const uint32_t r64 = d >= M ? 64u : (d >= 64 ? 64u : 64u % d);
      for (uint32_t c = 0; c < M; c += 64) {
        const uint32_t k = c + lane;
        if (k < M && d0 + k < blen) {
          const int32_t src = s + (int32_t)r;
          const uint32_t v = src >= 0 ? (uint32_t)S.tile[(uint32_t)src & (kB - 1)]
                                      : src_byte(A, sb + (int64_t)src, bad);
          S.tile[d0 + k] = (uint8_t)v;
        }
        r += r64;
        if (d < M && r >= d) r -= d;
      }
    };
    uint8_t* dummy = reinterpret_cast<uint8_t*>(&S.dummy[lane]);
    const uint32_t* tw = reinterpret_cast<const uint32_t*>(S.tile);
    for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
      const uint32_t a = c0 + lane;
      const bool have = a < cnt;
      const uint32_t aa = have ? a : c0;
      const uint32_t rng = Fr[aa];
      const uint32_t plo = rng & 63u, phi = (rng >> 8) & 63u;
      const uint64_t needm = have && phi > plo ? (1ull << phi) - (1ull << plo) : 0ull;
      const uint32_t pk = Fp[aa];
      const uint32_t dst = Fd[aa], len = Fl[aa];
      const int32_t s = (int32_t)(pk & 0xFFFFu) - 16384;
      const uint32_t d = (pk >> 16) & 0x7FFFu;
      const bool fast = d >= len && len <= kFastLen && s >= 0;
      bool pending = have;
      uint64_t done = ~__ballot(pending);
      for (uint32_t pass = 0; pass <= 64; pass++) {
        const bool ready = pending && (needm & ~done) == 0;
        const uint64_t m = __ballot(ready);
        if (!m) break;
        CLK_ADD(S, 10, 1);
        const bool rf = ready && fast;
        if (__ballot(rf)) {
          // source words covering [s, s + len), realigned to the source start
          const uint32_t w0 = (uint32_t)max(s, 0) >> 2, o = (uint32_t)max(s, 0) & 3u;
          uint32_t Wd[kFastLen / 4 + 1];
#pragma unroll
          for (uint32_t i = 0; i < kFastLen / 4 + 1; i++) Wd[i] = tw[min(w0 + i, kB / 4 - 1)];
          uint32_t Al[kFastLen / 4];
#pragma unroll
          for (uint32_t i = 0; i < kFastLen / 4; i++) Al[i] = __builtin_amdgcn_alignbyte(Wd[i + 1], Wd[i], o);
          const uint32_t lim = rf ? len : 0u;
#pragma unroll
          for (uint32_t g = 0; g < kFastLen / 4; g++) {
            if (!__ballot(4 * g < lim)) break;
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
              const uint32_t k = 4 * g + u;
              uint8_t* p = k < lim ? S.tile + dst + k : dummy + u;
              *p = (uint8_t)(Al[g] >> (8 * u));
            }
          }
        }
        uint64_t slow = __ballot(ready && !fast);
        const uint64_t c1_ = CLK_NOW();
        CLK_ADD(S, 11, __popcll(slow));
        while (slow) {                        // wave-uniform
          const uint32_t l = (uint32_t)__builtin_ctzll(slow);
          slow &= slow - 1;
          copy_match(c0 + l);
        }
        CLK_ADD(S, 12, CLK_NOW() - c1_);
        pending = pending && !ready;
        done |= m;
        // the next pass reads what this one wrote (LDS operations of a wave
        // are performed in order; the fence keeps the compiler from moving
        // the reads above the stores)
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      if (__ballot(pending)) bad = true;      // unreachable for a valid block
    }
    if (bad) S.err = 1;
    __builtin_amdgcn_s_setprio(1);
    CLK_ADD(S, 13, CLK_NOW() - c4_);
  } else if (wv != 0 && ov) {
    // the preparation has slack (it ends well before wave 0's passes): it
    // yields issue to the waves on their workgroups' critical paths
    __builtin_amdgcn_s_setprio(0);
    prep_ring(S, A, nb);
    __builtin_amdgcn_s_setprio(1);
    CLK_ADD1(S, 14, CLK_NOW() - c4_);
  }
  __syncthreads();
  const bool prepared = ov && uni(S.pok) != 0;
  CLK_ADD(S, 15, prepared ? 1 : 0);
  CLK_MARK(S, 7);
  if (S.err) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return false;
  }

  // ---- stage 5: tile -> HBM with 16-byte stores
  uint8_t* dst = A.addr ? reinterpret_cast<uint8_t*>(A.addr[b]) : A.out + sb;
  if (dst) {
    const uint32_t full = blen >> 4;
    const uint4* s4 = reinterpret_cast<const uint4*>(S.tile);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (uint32_t c = t; c < full; c += kWG) d4[c] = s4[c];
    for (uint32_t c = (full << 4) + t; c < blen; c += kWG) dst[c] = S.tile[c];
  }
  CLK_MARK(S, 8);
#ifdef LZ_STAGE_CLOCKS
  if (t == 0) S.clk[9] += 1;
#endif
  return prepared;
}


// Once per workgroup: literal LUT image into LDS, small-stream cumulative tables.
__device__ __forceinline__ void load_tables(Smem& S, const DevArgs& A) {
  const uint32_t t = threadIdx.x, wv = uni(t >> 6);
  // the LUT image (256-byte aligned in the workspace) straight into LDS
  static_assert(kLutLit % (4 * kWG) == 0, "whole LUT rounds");
#pragma unroll 1
  for (uint32_t i = 0; i < kLutLit / (4 * kWG); i++)
    lds_dma16(A.lut + 4 * (t + kWG * i), S.lut + 4 * (64 * wv + kWG * i));
  if (t < 3 * 64) {          // waves 0..2: one table each, 4 symbols per lane
    const uint32_t k = t >> 6, lane = t & 63;
    const uint8_t* tab = A.arc + A.off_tables + 512 * (k + 1);
    uint32_t f[4], sum = 0;
    for (int q = 0; q < 4; q++) {
      f[q] = (uint32_t)tab[2 * (4 * lane + q)] | ((uint32_t)tab[2 * (4 * lane + q) + 1] << 8);
      sum += f[q];
    }
    uint32_t incl = sum;
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= (uint32_t)d) incl += y;
    }
    uint32_t c = incl - sum;
    for (int q = 0; q < 4; q++) {
      S.cum[k][4 * lane + q] = (uint16_t)c;
      c += f[q];
    }
    if (lane == 63) S.cum[k][256] = (uint16_t)min(c, 65535u);
  }
  lds_dma_wait();                      // this wave's LUT rows, before the barrier
  __syncthreads();
  // bucket index of each short stream: bucket b starts at slot b << bs
  for (uint32_t e = t; e < 3 * 256; e += kWG) {
    const uint32_t k = e >> 8, b = e & 255, P = A.P[1 + k];
    const uint32_t bs = P > 8 ? P - 8 : 0u;
    if ((b << bs) < (1u << P)) S.bkt[k][b] = (uint8_t)search_sym(S.cum[k], b << bs);
  }
}

// Grid-wide barrier of a cooperative launch: arrivals are counted in one
// control word (reset before the launch); barrier k (k = 1, 2, ...) completes
// when nwg * k workgroups have arrived.  Agent-scope release before the
// arrival and acquire after the wait make the blocks decoded before the
// barrier visible to every workgroup after it.  A wait longer than the spin
// limit latches the watchdog and lets the kernel finish (status ECORRUPT).
__device__ __forceinline__ void grid_barrier(uint32_t* ctl, uint32_t target, uint32_t spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctl + kCtlTicket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t seen;
    for (uint32_t spins = 0;
         (seen = __hip_atomic_load(ctl + kCtlTicket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target; spins++) {
      if (spins >= spin_limit || ((spins & 255u) == 255u && watchdog_fired(ctl))) {
        watchdog(ctl, 4, target, 0, seen, target);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Per-level launches: a grid-stride slice of the level's queue; a workgroup
// without a block leaves before loading any table.  Persistent (one
// cooperative launch, every workgroup resident): the levels in order, each a
// grid-stride slice of qptr[L] .. qptr[L+1], a grid barrier before every
// non-empty level but the first.  decode_block has one call site, so the
// kernel's register budget is that of one copy of it.
__global__ void __launch_bounds__(kWG, 3) k_decode(DevArgs A) {   // 3 waves per SIMD: at most 168 VGPRs
  __shared__ Smem S;
  // issue priority: 1 by default, 2 for wave 0's in-block passes, 0 for the
  // next block's preparation by waves 1..3 (the one stage with slack)
  __builtin_amdgcn_s_setprio(1);
  const uint32_t t = threadIdx.x;
  uint32_t it = 0, qe = 0, L = 0, bars = 0;
  bool pending = false;       // (persistent) a non-empty level has been started
  if (!A.persistent) {
    uint32_t qb = A.q_begin;
    qe = A.q_end;
    if (A.qptr) {
      qb = A.qptr[A.q_begin];
      qe = A.qptr[A.q_end];
    }
    it = qb + blockIdx.x;
    if (it >= qe) return;
  }
#ifdef LZ_STAGE_CLOCKS
  if (t < kClkSlots) S.clk[t] = 0;
#endif
  bool tables = false;        // tables are loaded before the workgroup's first block
  bool prepared = false;      // the next block's stages 0 and 1 are done
  for (;;) {
    if (A.persistent) {
      while (it >= qe && L < kMaxLevels) {     // this workgroup's next block, in a later level
        const uint32_t b0 = A.qptr[L], b1 = A.qptr[L + 1];
        L++;
        if (b0 >= b1) continue;
        if (pending) grid_barrier(A.ctl, gridDim.x * ++bars, A.spin_limit);
        pending = true;
        it = b0 + blockIdx.x;
        qe = b1;
      }
    }
    if (it >= qe) break;
    if (!tables) {
      load_tables(S, A);
      __syncthreads();
      tables = true;
    }
    const uint32_t nit = it + gridDim.x;
    const uint32_t b = A.queue[it], nb = nit < qe ? A.queue[nit] : ~0u;
    if (!prepared) prep_tile(S, A, b);
    prepared = decode_block(S, A, b, nb);
    __syncthreads();
    it = nit;
  }
#ifdef LZ_STAGE_CLOCKS
  __syncthreads();
  if (t < kClkSlots) atomicAdd(reinterpret_cast<unsigned long long*>(A.ctl + kCtlClock) + t,
                               (unsigned long long)S.clk[t]);
#endif
}

// ---- setup kernels ---------------------------------------------------------

// Packed literal decode entry of slot u: symbol | f << 8 | (u - c_s) << 20.
__global__ void k_build_lut(const uint8_t* arc, uint64_t off_tables, uint32_t P, uint32_t* lut) {
  __shared__ uint32_t cum[257];
  __shared__ uint32_t fr[256];
  for (int s = threadIdx.x; s < 256; s += blockDim.x)
    fr[s] = (uint32_t)arc[off_tables + 2 * s] | ((uint32_t)arc[off_tables + 2 * s + 1] << 8);
  __syncthreads();
  if (threadIdx.x == 0) {
    cum[0] = 0;
    for (int s = 0; s < 256; s++) cum[s + 1] = cum[s] + fr[s];
  }
  __syncthreads();
  const uint32_t M = 1u << P;
  for (uint32_t u = threadIdx.x; u < kLutLit; u += blockDim.x) {
    if (cum[256] != M || u >= M) { lut[u] = 0; continue; }
    uint32_t lo = 0;
    for (uint32_t step = 128; step; step >>= 1)
      if (cum[lo + step] <= u) lo += step;
    lut[u] = lo | ((fr[lo] & 0xFFFu) << 8) | ((u - cum[lo]) << 20);
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

// Decode workgroups resident per compute unit (the cooperative grid is this
// times the CU count).
int lz_decode_occupancy(int* per_cu) {
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, reinterpret_cast<const void*>(k_decode),
                                                                    (int)kWG, 0);
  if (e != hipSuccess) return lz_fail(LZ_EDEVICE, "decode occupancy: %s", hipGetErrorString(e));
  return LZ_OK;
}

static DevArgs make_args(const lz_handle* h) {
  DevArgs A{};
  const ArchiveView& v = h->av;
  A.arc = v.base;
  A.n = v.n;
  A.off_tables = v.off_tables;
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
  hipLaunchKernelGGL(k_build_lut, dim3(1), dim3(256), 0, s, v.base, v.off_tables, v.prob_bits[0], h->ws.lut);
  const uint64_t nb = v.n_blocks;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(4096, (nb + 255) / 256 + 1);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, h->ws.flags, nb, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, h->ws.mark, nb, 0u);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, h->ws.addr, nb, 0ull);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, h->ws.ctl, (uint64_t)kCtlWords, 0u);
  return launch_ok("lz_open setup kernels");
}

// Persistent mode: one cooperative launch of every resident workgroup (the
// runtime refuses it rather than leave any workgroup waiting for a slot).
// Inside a stream capture the levels are launched one by one instead.
static int launch_persistent(lz_handle* h, DevArgs A, hipStream_t s, bool* done) {
  *done = false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return lz_fail(LZ_EDEVICE, "stream capture query failed");
  if (cs != hipStreamCaptureStatusNone) return LZ_OK;
  A.persistent = 1;
  void* args[] = {&A};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_decode), dim3(h->coop_grid),
                                                  dim3(kWG), args, 0, s);
  if (e != hipSuccess) return lz_fail(LZ_EDEVICE, "cooperative decode launch: %s", hipGetErrorString(e));
  *done = true;
  return LZ_OK;
}

int lz_launch_decode_all(lz_handle* h, uint8_t* out, hipStream_t s) {
  DevArgs A = make_args(h);
  A.queue = h->ws.queue;
  A.out = out;
  const size_t smem = 0;   // all LDS is static
  const uint32_t slots = (uint32_t)(h->n_cu * std::max(1u, h->tune.wg_per_cu));
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, h->ws.ctl);
  if (h->tune.sync_mode == 1) {
    A.qptr = h->ws.level_ptr;
    bool done = false;
    const int rc = launch_persistent(h, A, s, &done);
    if (rc || done) return rc ? rc : launch_ok("lz_decode_all");
  }
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
  return launch_ok("lz_decode_all");
}

// ---- verification: per-block FNV-1a-64 against the directory -----------------
namespace {

// Blocks b0 .. b0 + nb - 1 of the file, decoded at out (block b0 first): one
// thread per block hashes it with FNV-1a-64 and compares the hash with the
// directory's source hash.
__global__ void k_fnv_blocks(const uint8_t* arc, uint64_t off_dir, const uint8_t* out, uint64_t n,
                             uint32_t bl, uint64_t b0, uint64_t nb, uint64_t* hashes, uint32_t* ctl) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const uint64_t b = b0 + i;
  const uint64_t sb = b << bl, B = 1ull << bl;
  const uint64_t len = sb + B <= n ? B : n - sb;
  const uint8_t* src = out + (i << bl);
  uint64_t h = kFnvBasis;
  const uint4* p = reinterpret_cast<const uint4*>(src);
  uint64_t k = 0;
  for (; k + 16 <= len; k += 16) {
    const uint4 v = p[k >> 4];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int j = 0; j < 4; j++) h = (h ^ ((w[q] >> (8 * j)) & 0xFFu)) * kFnvPrime;
  }
  for (; k < len; k++) h = (h ^ src[k]) * kFnvPrime;
  hashes[i] = h;
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

int lz_launch_verify(lz_handle* h, const uint8_t* d_out, uint64_t b0, uint64_t nb, uint64_t* d_tree,
                     void* scratch, hipStream_t s) {
  uint64_t* hashes = reinterpret_cast<uint64_t*>(scratch);
  if (nb) {
    if ((uintptr_t)d_out & 15) return lz_fail(LZ_EINVAL, "lz_verify: output must be 16-byte aligned");
    hipLaunchKernelGGL(k_fnv_blocks, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, s, h->av.base,
                       h->av.off_dir, d_out, h->av.n, h->av.block_log2, b0, nb, hashes, h->ws.ctl);
  }
  if (d_tree) hipLaunchKernelGGL(k_fnv_tree, dim3(1), dim3(1), 0, s, hashes, nb, d_tree);
  return launch_ok("lz_verify");
}

// ---- FASTA regions: bases of a sequence gathered from its decoded bytes -------
namespace {

// out[i] = base start + i of a sequence whose first base is at byte `offset`
// of the file, W bases per line of LB bytes; tmp holds the file bytes from
// `first` on.
__global__ void k_region_gather(const uint8_t* tmp, uint64_t first, uint64_t offset, uint64_t start,
                                uint64_t nb, uint32_t W, uint32_t LB, uint8_t* out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nb;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = start + i;
    out[i] = tmp[offset + (k / W) * LB + k % W - first];
  }
}

}  // namespace

int lz_launch_region_gather(const uint8_t* tmp, uint64_t first, uint64_t offset, uint64_t start,
                            uint64_t nb, uint32_t W, uint32_t LB, uint8_t* out, hipStream_t s) {
  const uint32_t grid = (uint32_t)std::min<uint64_t>(4096, (nb + 255) / 256);
  hipLaunchKernelGGL(k_region_gather, dim3(grid), dim3(256), 0, s, tmp, first, offset, start, nb, W, LB, out);
  return launch_ok("lz_decode_region");
}

// ---- requests: ranges, read lookups, batches --------------------------------
//
// A batch is resolved by a fixed sequence of launches whose sizes are read on
// the device, so the sequence can be captured once and replayed:
//   begin   new request and completion epochs, counters cleared
//   spans   request -> [start, end) bytes (read id through the read index)
//   scan    exclusive prefix of lengths (output offsets) and of covering-block
//           counts (request, block) pairs; capacity check
//   mark    every covering block marked with the epoch and pushed on a list
//   closure worklist over the dependency lists: each pushed block pushes its
//           unmarked dependencies (transitive closure)
//   levels  counting sort of the closure by dependency level; each block gets
//           an address: straight into the output when it lies wholly inside an
//           aligned single range, else a scratch slot
//   decode  k_decode over the level-ordered closure (same body as whole-file)
//   gather  requested bytes of scratch-resident blocks copied to the output
namespace {

struct ReqArgs {
  const uint8_t* arc;
  uint64_t n, n_blocks, off_dir, off_dep_ptr, off_dep_idx, off_ridx, n_reads;
  uint32_t bl, mode, direct;
  uint64_t a0, b0;            // mode 0: the single range
  const int64_t* ids;         // mode 1: read ids
  const lz_request* reqs;     // mode 2: requests
  const uint32_t* d_n;        // mode 2: device request count
  uint64_t n_max;
  uint8_t* out;
  uint64_t cap;
  uint64_t* offsets;          // caller's offsets (n + 1) or null
  uint64_t* spans;            // scratch: 2 per request
  uint64_t* cnt_ptr;          // scratch: n + 1
  uint64_t* offs;             // scratch: n + 1
  uint8_t* slots;
  uint64_t max_slots;
  uint32_t* mark;
  uint64_t* addr;
  uint32_t* rqueue;
  uint32_t* rlevel_ptr;
  uint64_t* list;
  uint32_t* ctl;
};

__device__ __forceinline__ uint64_t* ctl64(uint32_t* ctl, uint32_t w) { return reinterpret_cast<uint64_t*>(ctl + w); }

__device__ __forceinline__ uint32_t aload(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// largest j in [0, n) with v[j] <= g (v nondecreasing, v[0] = 0)
__device__ __forceinline__ uint32_t find_req(const uint64_t* v, uint32_t n, uint64_t g) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (v[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Mark block b with the request epoch; push it on the closure list if this
// call marked it first.
__device__ __forceinline__ void mark_push(const ReqArgs& R, uint32_t b, uint32_t epoch) {
  const uint32_t old = __hip_atomic_fetch_max(R.mark + b, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (old >= epoch) return;
  const uint32_t i = __hip_atomic_fetch_add(R.ctl + kCtlListTail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(R.list + i, ((uint64_t)epoch << 32) | b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup.  First the address-table entries of the previous call's
// closure (still in the work list) are cleared, so that afterwards exactly the
// blocks of this call's closure have an address: a match whose source lies in
// any other block reads a null entry and fails as corrupt instead of following
// a pointer into a buffer of an earlier call.  Then the counters are reset.
__global__ void __launch_bounds__(256) k_req_begin(ReqArgs R) {
  const uint32_t t = threadIdx.x;
  const uint32_t prev = min(R.ctl[kCtlListTail], (uint32_t)R.n_blocks);
  for (uint32_t i = t; i < prev; i += blockDim.x) {
    const uint32_t b = (uint32_t)R.list[i];
    if (b < R.n_blocks) R.addr[b] = 0;
  }
  __syncthreads();
  if (t < 64) R.ctl[kCtlLevelCnt + t] = 0;
  if (t == 0) {
    R.ctl[kCtlREpoch] += 1;
    R.ctl[kCtlEpoch] += 1;
    R.ctl[kCtlTicket] = 0;
    R.ctl[kCtlListTail] = 0;
    R.ctl[kCtlListHead] = 0;
    R.ctl[kCtlListDone] = 0;
    R.ctl[kCtlSlots] = 0;
    uint64_t n = R.n_max;
    if (R.mode == 2) n = min((uint64_t)*R.d_n, R.n_max);
    R.ctl[kCtlNReq] = (uint32_t)n;
    *ctl64(R.ctl, kCtlTotal) = 0;
    *ctl64(R.ctl, kCtlPairs) = 0;
  }
}

__device__ __forceinline__ bool read_span(const ReqArgs& R, int64_t r, uint64_t& s, uint64_t& e) {
  if (!R.off_ridx || r < 0 || (uint64_t)r >= R.n_reads) return false;
  s = ld64(R.arc + R.off_ridx + 8ull * (uint64_t)r);
  e = ld64(R.arc + R.off_ridx + 8ull * (uint64_t)r + 8);
  return true;
}

__global__ void k_req_spans(ReqArgs R) {
  const uint32_t nreq = R.ctl[kCtlNReq];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nreq; j += gridDim.x * blockDim.x) {
    uint64_t s = 0, e = 0;
    bool ok = true;
    if (R.mode == 0) {
      s = R.a0;
      e = R.a0 + R.b0;
    } else if (R.mode == 1) {
      ok = read_span(R, R.ids[j], s, e);
    } else {
      const lz_request q = R.reqs[j];
      if (q.kind == 0) {
        ok = read_span(R, q.a, s, e);
      } else if (q.kind == 1 && q.a >= 0 && q.b >= 0 && (uint64_t)q.a <= R.n && (uint64_t)q.b <= R.n - (uint64_t)q.a) {
        s = (uint64_t)q.a;
        e = s + (uint64_t)q.b;
      } else {
        ok = false;
      }
    }
    if (!ok) {
      latch(R.ctl, kStRange);
      s = e = 0;
    }
    R.spans[2 * j] = s;
    R.spans[2 * j + 1] = e;
  }
}

// One workgroup of 1024 threads: exclusive prefix sums of output lengths and
// covering-block counts, in chunks of 1024 requests.
__global__ void __launch_bounds__(1024) k_req_scan(ReqArgs R) {
  __shared__ uint64_t wsum[2][16];
  const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t nreq = R.ctl[kCtlNReq];
  uint64_t carry_len = 0, carry_cnt = 0;
  for (uint32_t c0 = 0; c0 < nreq; c0 += 1024) {
    const uint32_t j = c0 + t;
    uint64_t len = 0, cnt = 0;
    if (j < nreq) {
      const uint64_t s = R.spans[2 * j], e = R.spans[2 * j + 1];
      len = e - s;
      cnt = e > s ? ((e - 1) >> R.bl) - (s >> R.bl) + 1 : 0;
    }
    uint64_t il = len, ic = cnt;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t yl = __shfl_up(il, d, 64), yc = __shfl_up(ic, d, 64);
      if (lane >= (uint32_t)d) { il += yl; ic += yc; }
    }
    if (lane == 63) { wsum[0][wv] = il; wsum[1][wv] = ic; }
    __syncthreads();
    uint64_t bl = 0, bc = 0, tl = 0, tc = 0;
    for (uint32_t q = 0; q < 16; q++) {
      if (q < wv) { bl += wsum[0][q]; bc += wsum[1][q]; }
      tl += wsum[0][q];
      tc += wsum[1][q];
    }
    if (j < nreq) {
      R.offs[j] = carry_len + bl + il - len;
      R.cnt_ptr[j] = carry_cnt + bc + ic - cnt;
      if (R.offsets) R.offsets[j] = carry_len + bl + il - len;
    }
    carry_len += tl;
    carry_cnt += tc;
    __syncthreads();
  }
  if (t == 0) {
    R.offs[nreq] = carry_len;
    R.cnt_ptr[nreq] = carry_cnt;
    if (R.offsets) R.offsets[nreq] = carry_len;
    *ctl64(R.ctl, kCtlTotal) = carry_len;
    if (carry_len > R.cap) {
      latch(R.ctl, kStCapacity);
      carry_cnt = 0;           // nothing is decoded or gathered
    }
    *ctl64(R.ctl, kCtlPairs) = carry_cnt;
  }
}

__global__ void k_req_mark(ReqArgs R) {
  const uint64_t pairs = *ctl64(R.ctl, kCtlPairs);
  const uint32_t nreq = R.ctl[kCtlNReq];
  const uint32_t epoch = R.ctl[kCtlREpoch];
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < pairs; g += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = find_req(R.cnt_ptr, nreq, g);
    const uint64_t b = (R.spans[2 * j] >> R.bl) + (g - R.cnt_ptr[j]);
    mark_push(R, (uint32_t)b, epoch);
  }
}

// Transitive closure over the dependency lists with a shared worklist.
// Control flow is uniform per wave (lanes of a wave cannot wait for each
// other): a wave takes 64 consecutive list indices, expands those already
// pushed (tail), and keeps the rest pending.  An expansion pushes the block's
// unmarked dependencies and then counts itself done with release order; with
// nothing ready, the wave loads done with acquire order and then tail: done ==
// tail means no entry is in flight and none can appear, so the pending indices
// stay empty and the wave stops.
__global__ void k_closure(ReqArgs R, uint32_t spin_limit) {
  const uint32_t lane = lane_id();
  const uint32_t epoch = aload(R.ctl + kCtlREpoch);
  for (;;) {
    uint32_t i0 = 0;
    if (lane == 0) i0 = __hip_atomic_fetch_add(R.ctl + kCtlListHead, 64u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    i0 = __shfl(i0, 0, 64);
    const uint32_t i = i0 + lane;
    bool pending = true;
    uint32_t spins = 0;
    while (__ballot(pending)) {
      const uint32_t tail = __shfl(aload(R.ctl + kCtlListTail), 0, 64);
      const bool ready = pending && i < tail;
      if (__ballot(ready)) {
        if (ready) {
          uint64_t v;
          uint32_t sp = 0;
          while (((v = __hip_atomic_load(R.list + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != epoch) {
            if (++sp > spin_limit) { watchdog(R.ctl, 2, i, (uint32_t)v, (uint32_t)(v >> 32), epoch); break; }
            __builtin_amdgcn_s_sleep(1);
          }
          const uint32_t b = (uint32_t)v;
          if ((v >> 32) == epoch) {
            const uint64_t d0 = ld64(R.arc + R.off_dep_ptr + 8ull * b), d1 = ld64(R.arc + R.off_dep_ptr + 8ull * (b + 1));
            for (uint64_t k = d0; k < d1; k++) mark_push(R, ld32(R.arc + R.off_dep_idx + 4 * k), epoch);
          }
          __hip_atomic_fetch_add(R.ctl + kCtlListDone, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          pending = false;
        }
        spins = 0;
        continue;
      }
      const uint32_t done = __shfl(__hip_atomic_load(R.ctl + kCtlListDone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT), 0, 64);
      const uint32_t tail2 = __shfl(aload(R.ctl + kCtlListTail), 0, 64);
      if (done == tail2 && !__ballot(pending && i < tail2)) return;   // pending indices past the end
      if (++spins > spin_limit) {
        if (lane == 0) watchdog(R.ctl, 3, i0, done, tail2, epoch);
        return;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

__device__ __forceinline__ uint32_t block_level(const ReqArgs& R, uint32_t b) {
  const uint8_t* e = R.arc + R.off_dir + (uint64_t)b * kDirEntry + 20;
  return min((uint32_t)e[0] | ((uint32_t)e[1] << 8), 63u);
}

__global__ void k_req_levels(ReqArgs R) {
  const uint32_t cnt = R.ctl[kCtlListTail];
  const uint64_t B = 1ull << R.bl;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t b = (uint32_t)R.list[i];
    atomicAdd(R.ctl + kCtlLevelCnt + block_level(R, b), 1u);
    const uint64_t sb = (uint64_t)b << R.bl, eb = min(sb + B, R.n);
    uint64_t a = 0;
    if (R.direct && sb >= R.a0 && eb <= R.a0 + R.b0 && ((sb - R.a0) & 15) == 0) {
      a = reinterpret_cast<uint64_t>(R.out + (sb - R.a0));
    } else {
      const uint32_t slot = atomicAdd(R.ctl + kCtlSlots, 1u);
      if (slot < R.max_slots) a = reinterpret_cast<uint64_t>(R.slots + (uint64_t)slot * B);
      else latch(R.ctl, kStCapacity);
    }
    R.addr[b] = a;
  }
}

__global__ void k_req_level_scan(ReqArgs R) {
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (uint32_t L = 0; L < 64; L++) {
      R.rlevel_ptr[L] = s;
      R.rlevel_ptr[65 + L] = s;
      s += R.ctl[kCtlLevelCnt + L];
    }
    R.rlevel_ptr[64] = s;
  }
}

__global__ void k_req_scatter(ReqArgs R) {
  const uint32_t cnt = R.ctl[kCtlListTail];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t b = (uint32_t)R.list[i];
    const uint32_t pos = atomicAdd(R.rlevel_ptr + 65 + block_level(R, b), 1u);
    R.rqueue[pos] = b;
  }
}

// Plan of a small request call in one workgroup of 1024 threads, the same
// steps as k_req_begin .. k_req_scatter without launches between them: clear
// the previous closure's addresses, spans and prefix sums of the requests,
// covering blocks marked and listed, the dependency closure expanded round by
// round (a round takes every listed entry not yet expanded; a block joins the
// list once, when its mark is raised to this call's epoch), then a counting
// sort of the closure by level with each block's address.
constexpr uint32_t kPlanWG = 1024;

__global__ void __launch_bounds__(kPlanWG) k_req_plan(ReqArgs R) {
  __shared__ uint64_t wsum[2][kPlanWG / 64];
  __shared__ uint32_t lvl_cnt[64], lvl_cur[64];
  __shared__ uint32_t s_tail, s_slots, s_nreq, s_epoch;
  __shared__ uint64_t s_pairs;
  const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // begin: the previous call's closure loses its addresses; new epochs
  {
    const uint32_t prev = min(R.ctl[kCtlListTail], (uint32_t)R.n_blocks);
    for (uint32_t i = t; i < prev; i += kPlanWG) {
      const uint32_t b = (uint32_t)R.list[i];
      if (b < R.n_blocks) R.addr[b] = 0;
    }
  }
  if (t < 64) lvl_cnt[t] = 0;
  if (t == 0) {
    uint64_t n = R.n_max;
    if (R.mode == 2) n = min((uint64_t)*R.d_n, R.n_max);
    s_nreq = (uint32_t)n;
    s_tail = 0;
    s_slots = 0;
  }
  __syncthreads();
  if (t == 0) {
    s_epoch = R.ctl[kCtlREpoch] + 1;
    R.ctl[kCtlREpoch] = s_epoch;
    R.ctl[kCtlEpoch] += 1;
    R.ctl[kCtlTicket] = 0;
    R.ctl[kCtlListHead] = 0;
    R.ctl[kCtlListDone] = 0;
    R.ctl[kCtlNReq] = s_nreq;
  }
  __syncthreads();
  const uint32_t epoch = s_epoch;
  const uint32_t nreq = s_nreq;
  // spans, output offsets and covering-block counts, 1024 requests a round
  uint64_t carry_len = 0, carry_cnt = 0;
  for (uint32_t c0 = 0; c0 < nreq; c0 += kPlanWG) {
    const uint32_t j = c0 + t;
    uint64_t s0 = 0, e0 = 0;
    if (j < nreq) {
      bool ok = true;
      if (R.mode == 0) {
        s0 = R.a0;
        e0 = R.a0 + R.b0;
      } else if (R.mode == 1) {
        ok = read_span(R, R.ids[j], s0, e0);
      } else {
        const lz_request q = R.reqs[j];
        if (q.kind == 0) {
          ok = read_span(R, q.a, s0, e0);
        } else if (q.kind == 1 && q.a >= 0 && q.b >= 0 && (uint64_t)q.a <= R.n && (uint64_t)q.b <= R.n - (uint64_t)q.a) {
          s0 = (uint64_t)q.a;
          e0 = s0 + (uint64_t)q.b;
        } else {
          ok = false;
        }
      }
      if (!ok) {
        latch(R.ctl, kStRange);
        s0 = e0 = 0;
      }
      R.spans[2 * j] = s0;
      R.spans[2 * j + 1] = e0;
    }
    const uint64_t len = e0 - s0;
    const uint64_t cnt = e0 > s0 ? ((e0 - 1) >> R.bl) - (s0 >> R.bl) + 1 : 0;
    uint64_t il = len, ic = cnt;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t yl = __shfl_up(il, d, 64), yc = __shfl_up(ic, d, 64);
      if (lane >= (uint32_t)d) { il += yl; ic += yc; }
    }
    if (lane == 63) { wsum[0][wv] = il; wsum[1][wv] = ic; }
    __syncthreads();
    uint64_t bl = 0, bc = 0, tl = 0, tc = 0;
    for (uint32_t q = 0; q < kPlanWG / 64; q++) {
      if (q < wv) { bl += wsum[0][q]; bc += wsum[1][q]; }
      tl += wsum[0][q];
      tc += wsum[1][q];
    }
    if (j < nreq) {
      R.offs[j] = carry_len + bl + il - len;
      R.cnt_ptr[j] = carry_cnt + bc + ic - cnt;
      if (R.offsets) R.offsets[j] = carry_len + bl + il - len;
    }
    carry_len += tl;
    carry_cnt += tc;
    __syncthreads();
  }
  if (t == 0) {
    R.offs[nreq] = carry_len;
    R.cnt_ptr[nreq] = carry_cnt;
    if (R.offsets) R.offsets[nreq] = carry_len;
    *ctl64(R.ctl, kCtlTotal) = carry_len;
    uint64_t pairs = carry_cnt;
    if (carry_len > R.cap) {
      latch(R.ctl, kStCapacity);
      pairs = 0;                 // nothing is decoded or gathered
    }
    *ctl64(R.ctl, kCtlPairs) = pairs;
    s_pairs = pairs;
  }
  __syncthreads();
  // covering blocks: marked with this epoch and listed once each
  const uint64_t pairs = s_pairs;
  auto push = [&](uint32_t b) {
    const uint32_t old = __hip_atomic_fetch_max(R.mark + b, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old >= epoch) return;
    const uint32_t i = atomicAdd(&s_tail, 1u);
    if (i < R.n_blocks) R.list[i] = ((uint64_t)epoch << 32) | b;
  };
  for (uint64_t g = t; g < pairs; g += kPlanWG) {
    const uint32_t j = find_req(R.cnt_ptr, nreq, g);
    push((uint32_t)((R.spans[2 * j] >> R.bl) + (g - R.cnt_ptr[j])));
  }
  __syncthreads();
  // dependency closure, one round per pass over the entries listed so far.
  // Every thread reads the round's tail between two barriers, before anyone
  // pushes in this round: a wave reading it after another wave's pushes would
  // see a longer list, and threads leaving the loop in different rounds would
  // meet at different barriers.
  uint32_t head = 0;
  for (uint32_t round = 0; round <= R.n_blocks; round++) {
    const uint32_t tail = min(s_tail, (uint32_t)R.n_blocks);
    __syncthreads();
    if (head >= tail) break;
    for (uint32_t i = head + t; i < tail; i += kPlanWG) {
      const uint32_t b = (uint32_t)R.list[i];
      const uint64_t d0 = ld64(R.arc + R.off_dep_ptr + 8ull * b), d1 = ld64(R.arc + R.off_dep_ptr + 8ull * (b + 1));
      for (uint64_t k = d0; k < d1; k++) push(ld32(R.arc + R.off_dep_idx + 4 * k));
    }
    head = tail;
    __syncthreads();
  }
  const uint32_t cnt = min(s_tail, (uint32_t)R.n_blocks);
  // levels and addresses: straight into the output for a block wholly inside
  // an aligned single range, else a scratch slot
  const uint64_t B = 1ull << R.bl;
  for (uint32_t i = t; i < cnt; i += kPlanWG) {
    const uint32_t b = (uint32_t)R.list[i];
    atomicAdd(&lvl_cnt[block_level(R, b)], 1u);
    const uint64_t sb = (uint64_t)b << R.bl, eb = min(sb + B, R.n);
    uint64_t a = 0;
    if (R.direct && sb >= R.a0 && eb <= R.a0 + R.b0 && ((sb - R.a0) & 15) == 0) {
      a = reinterpret_cast<uint64_t>(R.out + (sb - R.a0));
    } else {
      const uint32_t slot = atomicAdd(&s_slots, 1u);
      if (slot < R.max_slots) a = reinterpret_cast<uint64_t>(R.slots + (uint64_t)slot * B);
      else latch(R.ctl, kStCapacity);
    }
    R.addr[b] = a;
  }
  __syncthreads();
  if (t < 64) {                                 // exclusive scan of the 64 level counts
    const uint32_t c = lvl_cnt[t];
    uint32_t incl = c;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (t >= (uint32_t)d) incl += y;
    }
    R.rlevel_ptr[t] = incl - c;
    R.rlevel_ptr[65 + t] = incl - c;
    lvl_cur[t] = incl - c;
    if (t == 63) R.rlevel_ptr[64] = incl;
  }
  __syncthreads();
  for (uint32_t i = t; i < cnt; i += kPlanWG) {
    const uint32_t b = (uint32_t)R.list[i];
    R.rqueue[atomicAdd(&lvl_cur[block_level(R, b)], 1u)] = b;
  }
  if (t == 0) {
    R.ctl[kCtlListTail] = cnt;
    R.ctl[kCtlSlots] = s_slots;
    if (s_tail > R.n_blocks) latch(R.ctl, kStCorrupt);
  }
}

// One workgroup per (request, covering block) pair: copy the requested part
// of a block that was decoded into a scratch slot.
__global__ void k_req_gather(ReqArgs R) {
  const uint64_t pairs = *ctl64(R.ctl, kCtlPairs);
  const uint32_t nreq = R.ctl[kCtlNReq];
  const uint64_t B = 1ull << R.bl;
  for (uint64_t g = blockIdx.x; g < pairs; g += gridDim.x) {
    const uint32_t j = find_req(R.cnt_ptr, nreq, g);
    const uint64_t s = R.spans[2 * j], e = R.spans[2 * j + 1];
    const uint64_t b = (s >> R.bl) + (g - R.cnt_ptr[j]);
    const uint64_t a = R.addr[b];
    if (!a) continue;
    const uint64_t sb = b << R.bl, eb = min(sb + B, R.n);
    const uint64_t lo = max(sb, s), hi = min(eb, e);
    if (hi <= lo) continue;
    uint8_t* dst = R.out + R.offs[j] + (lo - s);
    const uint8_t* src = reinterpret_cast<const uint8_t*>(a) + (lo - sb);
    if (src == dst) continue;   // decoded in place
    for (uint64_t q = threadIdx.x; q < hi - lo; q += blockDim.x) dst[q] = src[q];
  }
}

}  // namespace

int lz_launch_requests(lz_handle* h, const lz_request* d_reqs, const uint32_t* d_n, uint64_t n_max,
                       uint64_t single_off, uint64_t single_len, const int64_t* d_ids,
                       uint8_t* d_out, uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                       uint64_t scratch_len, hipStream_t s) {
  const ArchiveView& v = h->av;
  ReqArgs R{};
  R.arc = v.base;
  R.n = v.n;
  R.n_blocks = v.n_blocks;
  R.off_dir = v.off_dir;
  R.off_dep_ptr = v.off_dep_ptr;
  R.off_dep_idx = v.off_dep_idx;
  R.off_ridx = v.kind == 1 ? v.off_ridx : 0;
  R.n_reads = v.n_reads;
  R.bl = v.block_log2;
  R.mode = d_reqs ? 2u : (d_ids ? 1u : 0u);
  R.a0 = single_off;
  R.b0 = single_len;
  R.ids = d_ids;
  R.reqs = d_reqs;
  R.d_n = d_n;
  R.n_max = n_max;
  R.out = d_out;
  R.cap = cap;
  R.offsets = d_offsets;
  // scratch: spans, block-count prefix, output prefix, then 16 KiB slots
  const uint64_t B = 1ull << v.block_log2;
  uint8_t* sc = reinterpret_cast<uint8_t*>(d_scratch);
  if (!sc || ((uintptr_t)sc & 255)) return lz_fail(LZ_EINVAL, "request scratch must be 256-byte aligned");
  const uint64_t spans_b = 16 * n_max, ptr_b = 8 * (n_max + 1);
  const uint64_t slots_off = (spans_b + 2 * ptr_b + 255) & ~255ull;
  if (scratch_len < slots_off) return lz_fail(LZ_ECAPACITY, "request scratch needs at least %llu bytes", (unsigned long long)slots_off);
  R.spans = reinterpret_cast<uint64_t*>(sc);
  R.cnt_ptr = reinterpret_cast<uint64_t*>(sc + spans_b);
  R.offs = reinterpret_cast<uint64_t*>(sc + spans_b + ptr_b);
  R.slots = sc + slots_off;
  R.max_slots = (scratch_len - slots_off) / B;
  R.direct = (R.mode == 0 && ((uintptr_t)d_out & 15) == 0) ? 1u : 0u;
  R.mark = h->ws.mark;
  R.addr = h->ws.addr;
  R.rqueue = h->ws.rqueue;
  R.rlevel_ptr = h->ws.rlevel_ptr;
  R.list = h->ws.list;
  R.ctl = h->ws.ctl;
  const uint32_t spin = h->tune.spin_limit ? h->tune.spin_limit : (1u << 20);
  const uint32_t g_req = (uint32_t)std::min<uint64_t>(1024, (n_max + 255) / 256);
  // small calls are planned by one workgroup (one launch instead of eight):
  // at most plan_blocks covering blocks expected (a range, reads at two
  // blocks each, batches at 256 blocks a request)
  const uint64_t Bs = 1ull << v.block_log2, pb = h->tune.plan_blocks ? h->tune.plan_blocks : 4096;
  const bool small = R.mode == 0 ? single_len / Bs + 2 <= pb
                   : R.mode == 1 ? n_max * (v.max_record_len / Bs + 2) <= pb
                                 : n_max * 256 <= pb;
  const uint32_t g_wide = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (v.n_blocks + 255) / 256));
  if (small) {
    hipLaunchKernelGGL(k_req_plan, dim3(1), dim3(kPlanWG), 0, s, R);
  } else {
    hipLaunchKernelGGL(k_req_begin, dim3(1), dim3(256), 0, s, R);
    hipLaunchKernelGGL(k_req_spans, dim3(g_req), dim3(256), 0, s, R);
    hipLaunchKernelGGL(k_req_scan, dim3(1), dim3(1024), 0, s, R);
    hipLaunchKernelGGL(k_req_mark, dim3(g_wide), dim3(256), 0, s, R);
    hipLaunchKernelGGL(k_closure, dim3(std::min<uint32_t>(64, g_wide)), dim3(256), 0, s, R, spin);
    hipLaunchKernelGGL(k_req_levels, dim3(g_wide), dim3(256), 0, s, R);
    hipLaunchKernelGGL(k_req_level_scan, dim3(1), dim3(64), 0, s, R);
    hipLaunchKernelGGL(k_req_scatter, dim3(g_wide), dim3(256), 0, s, R);
  }
  // decode the closure in level order (one cooperative launch, or one launch per level)
  DevArgs A = make_args(h);
  A.queue = h->ws.rqueue;
  A.qptr = h->ws.rlevel_ptr;
  A.addr = h->ws.addr;
  A.out = d_out;
  const uint32_t slots = (uint32_t)(h->n_cu * std::max(1u, h->tune.wg_per_cu));
  const uint32_t grid = (uint32_t)std::min<uint64_t>(slots, std::max<uint64_t>(1, v.n_blocks));
  bool done = false;
  if (h->tune.req_sync_mode == 1) {
    const int rc = launch_persistent(h, A, s, &done);
    if (rc) return rc;
  }
  if (!done) {
    for (uint32_t L = 0; L < v.n_levels; L++) {
      A.q_begin = L;
      A.q_end = L + 1;
      hipLaunchKernelGGL(k_decode, dim3(grid), dim3(kWG), 0, s, A);
    }
  }
  hipLaunchKernelGGL(k_req_gather, dim3(g_wide), dim3(256), 0, s, R);
  return launch_ok("request decode");
}
