// Device decoder for container format v2 on gfx950 (CDNA4, wave64).
//
// One workgroup of 256 threads (4 waves) decodes one block at a time:
//   1. waves 0..2 decode the command (CMD), match-length (MLEN) and offset
//      (OFF) streams, one each, reading rANS words straight from HBM;
//   2. block-wide exclusive scans turn literal-run and match lengths into
//      literal and output positions (command placement);
//   3. the literal stream's 64-lane groups are decoded by one wave each and
//      every literal is written straight to its output position in an LDS tile;
//   4. matches whose source lies wholly in earlier blocks are copied in
//      parallel; then the remaining matches are copied in order, each with
//      out[p+k] = out[OF + (k mod (p-OF))], the byte-sequential overlap rule
//      out[p+k] = out[OF+k] unrolled, so all bytes of a match go at once;
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
constexpr uint32_t kLutLit = 1u << kMaxPLit;      // 4096 packed literal entries
constexpr uint32_t kL = 1u << 16;                 // rANS state lower bound

// All LDS is static (about 51.8 KB, three workgroups per CU): literal LUT,
// output tile, small-stream cumulative tables, per-sequence tables.
struct Smem {
  uint32_t lut[kLutLit];
  alignas(16) uint8_t tile[kB];
  uint16_t cum[3][257];        // CMD, MLEN, OFF cumulative frequencies
  uint8_t bkt[3][256];         // per stream: symbol owning the first slot of each bucket
  uint16_t lit[kMaxSeq + 1];   // LL values, then exclusive scan of LL ([ns] = n_lit)
  uint16_t out[kMaxSeq + 1];   // ML values, then exclusive scan of LL+ML ([ns] = block length)
  uint32_t oflo[kMaxSeq];      // absolute source offsets, low 32 bits
  uint8_t ofhi[kMaxSeq + 3];   // bits 32..39
  uint16_t intl[kMaxSeq];      // matches whose source touches the block itself
  uint8_t plist[64];           // dependent matches of one pass (chunk-relative)
  uint32_t ppk[64], pdl[64];   // their packed source/period and destination | length << 16
  uint16_t ring[kWaves][256];  // rANS words staged per wave (two 128-word slices)
  uint32_t ringe[kWaves][256]; // literal stream: table entry of each staged word's slot
  uint32_t scan[kWaves];
  uint32_t item, err, nint;
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

// One stream record, parsed by every thread from global memory (uniform).
struct Stream {
  uint32_t mode, csym, K, n, nw, blen, body;
};

// Parse and check the record at *off of a block payload; advances *off.
// Parses one stream record header from the LDS copy `hp` of the first hlen
// payload bytes; records end within plen.  With `staged` the whole record must
// lie in the copy (the short streams are decoded from it).
__device__ __forceinline__ bool parse_stream(const uint8_t* hp, uint32_t hlen, uint32_t plen,
                                             uint32_t* off, uint32_t want, uint32_t maxK,
                                             bool staged, Stream& s) {
  if (*off + 16 > hlen) return false;
  const uint8_t* h = hp + *off;
  s.mode = h[0];
  s.csym = h[1];
  s.K = (uint32_t)h[2] | ((uint32_t)h[3] << 8);
  s.n = ld32(h + 4);
  s.nw = ld32(h + 8);
  s.blen = ld32(h + 12);
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
      uint64_t sum = 0;
      for (uint32_t g = 0; g < G; g++) sum += ld32(hp + s.body + 4 * s.K + 4 * g);
      if (sum != s.nw) return false;
      break;
    }
    default: return false;
  }
  *off = s.body + ((s.blen + 15u) & ~15u);
  return true;
}

// Decode the symbols of 64-lane group g of a rANS stream with one wave.
// `body` is the record body in global memory (states, per-group word counts,
// words).  `sym(u)` maps slot u to symbol | f << 8 | (u - c_s) << 20 and
// `out(i, s)` consumes symbol i.  The group's 16-bit words are staged through
// the wave's LDS ring (two 128-word slices, the next slice loading into
// registers meanwhile), so a lane needing word idx reads it from LDS.
// True if every state ends at 2^16 and every word of the group was read.
template <class Sym, class Out>
__device__ bool rans_group(const uint8_t* body, const Stream& s, uint32_t g, uint32_t P,
                           uint16_t* ring, Sym&& sym, Out&& out) {
  const uint32_t lane = lane_id();
  const uint32_t K = s.K, n = s.n, G = (K + 63) >> 6;
  const uint32_t k = (g << 6) + lane;
  const bool lane_ok = k < K;
  uint32_t woff = 0, nwg = 0;
  for (uint32_t q = 0; q < G; q++) {
    const uint32_t c = ld32(body + 4 * K + 4 * q);
    if (q < g) woff += c;
    if (q == g) nwg = c;
  }
  // Word loads are unconditional: an index past the group's end reads the
  // group's last word (or, for a group without words, the first state), so
  // every load stays inside the record; a corrupt stream that consumes more
  // words than the group holds fails the end check (pos == nwg).
  const uint16_t* W = nwg ? reinterpret_cast<const uint16_t*>(body + 4 * K + 4 * G) + woff
                          : reinterpret_cast<const uint16_t*>(body);
  const uint32_t lastw = nwg ? nwg - 1 : 0;
  auto ldw = [&](uint32_t idx) -> uint32_t { return (uint32_t)W[min(idx, lastw)]; };
  uint32_t x = lane_ok ? ld32(body + 4 * k) : kL;
  bool ok = x >= kL && woff + nwg <= s.nw;
  // Ring of two 128-word slices: with s = pos / 128, slices s and s+1 are in
  // the ring and slice s+2 is in flight in registers (pa, pb).
  {
    const uint32_t a0 = ldw(lane), a1 = ldw(64 + lane), a2 = ldw(128 + lane), a3 = ldw(192 + lane);
    ring[lane] = (uint16_t)a0;
    ring[64 + lane] = (uint16_t)a1;
    ring[128 + lane] = (uint16_t)a2;
    ring[192 + lane] = (uint16_t)a3;
  }
  uint32_t pa = ldw(256 + lane), pb = ldw(320 + lane);
  uint32_t pos = 0;
  // lane k decodes the run of consecutive symbols starting at
  // k*full + min(k, extra): full = n / K symbols, one more for the first
  // extra = n mod K lanes
  const uint32_t full = n / K, extra = n - full * K;
  const uint32_t mask = (1u << P) - 1;
  uint32_t i = k * full + min(k, extra);
  auto round = [&](bool act) {
    if (act) {
      const uint32_t e = sym(x & mask);
      x = __umul24((e >> 8) & 0xFFFu, x >> P) + (e >> 20);
      out(i, e & 0xFFu);
    }
    i += 1;
    const bool need = act && x < kL;
    const uint64_t bal = __ballot(need);
    if (bal) {
      if (need) x = (x << 16) | (uint32_t)ring[(pos + mbcnt(bal)) & 255];
      const uint32_t s0 = pos >> 7;
      pos += (uint32_t)__popcll(bal);
      if ((pos >> 7) != s0) {          // entered slice s0+1: stage s0+2, fetch s0+3
        __builtin_amdgcn_wave_barrier();   // after every lane's read of slice s0
        uint16_t* d = ring + ((s0 & 1) << 7) + lane;
        d[0] = (uint16_t)pa;
        d[64] = (uint16_t)pb;
        const uint32_t b3 = (s0 + 3) << 7;
        pa = ldw(b3 + lane);
        pb = ldw(b3 + 64 + lane);
      }
    }
  };
  // rounds in which every lane of the stream decodes, then the partial one
  for (uint32_t r = 0; r < full; r++) round(lane_ok);
  if (extra) round(lane_ok && k < extra);
  ok = ok && (!lane_ok || x == kL) && pos == nwg;
  return __ballot(!ok) == 0;
}

// The literal stream's group decode: the same symbols, words and checks as
// rans_group, with the next table lookup of a renormalising lane folded into
// its word read.  After x = (x << 16) | w the next slot is w mod 2^P (P <= 12),
// so every word staged into the ring carries the table entry of that slot.  A
// round then makes one LDS round trip: lanes that take a word read the word
// and its entry, the others look up their new slot, in the same wait.
// `out(i, s, act)` is called by every lane of the wave each round; only lanes
// with act set hold symbol i.
template <class Out>
__device__ bool rans_lit(const uint8_t* body, const Stream& s, uint32_t g, uint32_t P,
                         const uint32_t* lut, uint16_t* ring, uint32_t* ringe, Out&& out) {
  const uint32_t lane = lane_id();
  const uint32_t K = s.K, n = s.n, G = (K + 63) >> 6;
  const uint32_t k = (g << 6) + lane;
  const bool lane_ok = k < K;
  uint32_t woff = 0, nwg = 0;
  for (uint32_t q = 0; q < G; q++) {
    const uint32_t c = ld32(body + 4 * K + 4 * q);
    if (q < g) woff += c;
    if (q == g) nwg = c;
  }
  // unconditional word loads, clamped into the group as in rans_group
  const uint16_t* W = nwg ? reinterpret_cast<const uint16_t*>(body + 4 * K + 4 * G) + woff
                          : reinterpret_cast<const uint16_t*>(body);
  const uint32_t lastw = nwg ? nwg - 1 : 0;
  auto ldw = [&](uint32_t idx) -> uint32_t { return (uint32_t)W[min(idx, lastw)]; };
  const uint32_t mask = (1u << P) - 1;
  uint32_t x = lane_ok ? ld32(body + 4 * k) : kL;
  bool ok = x >= kL && woff + nwg <= s.nw;
  // ring of two 128-word slices as in rans_group; slice s+2 waits in pa, pb
  {
    uint32_t a[4];
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) a[q] = ldw(64 * q + lane);
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
      ring[64 * q + lane] = (uint16_t)a[q];
      ringe[64 * q + lane] = lut[a[q] & mask];
    }
  }
  uint32_t pa = ldw(256 + lane), pb = ldw(320 + lane);
  uint32_t e = lut[x & mask];
  uint32_t pos = 0;
  const uint32_t full = n / K, extra = n - full * K;
  uint32_t i = k * full + min(k, extra);
  // One round.  Both reads are issued by every lane (a lane without a word
  // reads a word it ignores; a lane with one takes its entry from the ring
  // instead of the table), then the symbol's tile store, so the next round
  // waits for the reads alone.
  auto round = [&](bool act) {
    const uint32_t xd = __umul24((e >> 8) & 0xFFFu, x >> P) + (e >> 20);
    const uint32_t sym = e & 0xFFu;
    if (act) x = xd;
    const bool need = act && x < kL;
    const uint64_t bal = __ballot(need);
    const uint32_t q = (pos + mbcnt(bal)) & 255;
    const uint32_t w = ring[q];
    e = need ? ringe[q] : lut[x & mask];
    out(i, sym, act);
    i += 1;
    x = need ? (x << 16) | w : x;
    if (bal) {
      const uint32_t s0 = pos >> 7;
      pos += (uint32_t)__popcll(bal);
      if ((pos >> 7) != s0) {          // entered slice s0+1: stage s0+2, fetch s0+3
        __builtin_amdgcn_wave_barrier();   // after every lane's read of slice s0
        const uint32_t ea = lut[pa & mask], eb = lut[pb & mask];
        const uint32_t d = ((s0 & 1) << 7) + lane;
        ring[d] = (uint16_t)pa;
        ring[d + 64] = (uint16_t)pb;
        ringe[d] = ea;
        ringe[d + 64] = eb;
        const uint32_t b3 = (s0 + 3) << 7;
        pa = ldw(b3 + lane);
        pb = ldw(b3 + 64 + lane);
      }
    }
  };
  if ((g << 6) + 64 <= K) {
    for (uint32_t r = 0; r < full; r++) round(true);   // every lane of the group decodes
  } else {
    for (uint32_t r = 0; r < full; r++) round(lane_ok);
  }
  if (extra) round(lane_ok && k < extra);
  ok = ok && (!lane_ok || x == kL) && pos == nwg;
  return __ballot(!ok) == 0;
}

// Source byte at absolute position a (an earlier block): direct mode reads the
// whole-file output; request mode goes through the per-block address table.
__device__ __forceinline__ uint32_t src_byte(const DevArgs& A, uint64_t a, bool& bad) {
  if (!A.addr) return A.out[a];
  const uint64_t base = A.addr[a >> A.bl];
  if (!base) { bad = true; return 0; }
  return reinterpret_cast<const uint8_t*>(base)[a & ((1ull << A.bl) - 1)];
}

// Block-wide exclusive scan of v; *total receives the sum.
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
    const uint32_t s = S.scan[q];
    if (q < (int)wv) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

// Small-stream symbol lookup: binary search of slot u in a 257-entry
// cumulative table; returns symbol | f << 8 | (u - c_s) << 20.
__device__ __forceinline__ uint32_t search_sym(const uint16_t* cum, uint32_t u) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = 128; step; step >>= 1)
    if (cum[lo + step] <= u) lo += step;
  return lo;
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

// Decode block b into the LDS tile and store it.  Every loop below is bounded
// by values read from global memory (directory, stream headers).
__device__ void decode_block(Smem& S, const DevArgs& A, uint32_t b) {
  const uint32_t t = threadIdx.x, wv = t >> 6, lane = lane_id();
  const uint64_t B = 1ull << A.bl;
  const uint64_t sb = (uint64_t)b << A.bl;
  const uint32_t blen = (uint32_t)((sb + B <= A.n) ? B : A.n - sb);
  const uint8_t* de = A.arc + A.off_dir + (uint64_t)b * kDirEntry;
  const uint64_t poff = ld64(de);
  const uint32_t plen = ld32(de + 8), ns = ld32(de + 12), nlit = ld32(de + 16);
  const uint8_t* pay = A.arc + A.off_payload + poff;

  // The first min(plen, 16 KiB) payload bytes are copied into the tile (free
  // until stage 3) with one round of 16-byte loads: the stream headers and
  // the short streams CMD, MLEN, OFF (at most about 9.3 KB with their headers
  // for 1025 sequences) are read from there; the literal stream from HBM.
  const uint32_t hlen = min(plen, kB);
  {
    const uint4* src4 = reinterpret_cast<const uint4*>(pay);
    uint4* dst4 = reinterpret_cast<uint4*>(S.tile);
    for (uint32_t c = t; c < (hlen >> 4); c += kWG) dst4[c] = src4[c];
    if (t < (hlen & 15u)) S.tile[(hlen & ~15u) + t] = pay[(hlen & ~15u) + t];
  }
  __syncthreads();
  const uint8_t* hp = S.tile;

  // stream records: CMD, MLEN, OFF, LIT (every thread parses the same bytes)
  Stream sc, sm, so, sl;
  uint32_t off = 0;
  bool ok = ns >= 1 && ns <= kMaxSeq && nlit <= blen && (poff & 15) == 0;
  ok = ok && parse_stream(hp, hlen, plen, &off, 2 * ns, A.seq_lanes, true, sc);
  ok = ok && parse_stream(hp, hlen, plen, &off, 2 * ns, A.seq_lanes, true, sm);
  ok = ok && parse_stream(hp, hlen, plen, &off, A.w * ns, A.seq_lanes, true, so);
  ok = ok && parse_stream(hp, hlen, plen, &off, nlit, A.lit_lanes, false, sl);
  if (!ok) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return;
  }

  // ---- stage 1: CMD -> lit[] (LL), MLEN -> out[] (ML), OFF -> oflo/ofhi
  for (uint32_t j = t; j < ns; j += kWG) { S.oflo[j] = 0; S.ofhi[j] = 0; }
  if (t == 0) { S.err = 0; S.nint = 0; }
  __syncthreads();
  if (wv < 3) {
    const Stream& s = wv == 0 ? sc : (wv == 1 ? sm : so);
    const uint16_t* cum = S.cum[wv];
    const uint32_t bs = A.P[1 + wv] > 8 ? A.P[1 + wv] - 8 : 0u;
    uint8_t* dst8 = wv == 0 ? reinterpret_cast<uint8_t*>(S.lit) : reinterpret_cast<uint8_t*>(S.out);
    auto put = [&](uint32_t i, uint32_t v) {
      uint32_t plane = 0, idx = i;
      while (idx >= ns && plane < 7) { idx -= ns; plane++; }
      if (wv < 2) {
        dst8[2 * idx + plane] = (uint8_t)v;
      } else if (plane < 4) {
        reinterpret_cast<uint8_t*>(S.oflo)[4 * idx + plane] = (uint8_t)v;
      } else {
        S.ofhi[idx] = (uint8_t)v;
      }
    };
    bool okw = true;
    if (s.mode == kModeRans) {
      okw = rans_group(hp + s.body, s, 0, A.P[1 + wv], S.ring[wv],
                       [&](uint32_t u) { return bucket_sym(cum, S.bkt[wv], bs, u); }, put);
    } else if (s.mode == kModeRaw) {
      const uint8_t* src = hp + s.body;
      for (uint32_t i = lane; i < s.n; i += 64) put(i, src[i]);
    } else if (s.mode == kModeConst) {
      for (uint32_t i = lane; i < s.n; i += 64) put(i, s.csym);
    }
    if (!okw && lane == 0) S.err = 1;
  }
  __syncthreads();

  // ---- stage 2: command placement; in-place exclusive scans of LL and LL+ML
  {
    const uint32_t per = (ns + kWG - 1) / kWG;
    const uint32_t j0 = min(ns, t * per), j1 = min(ns, j0 + per);
    uint32_t ll[5], ml[5];
    uint32_t sl_ = 0, so_ = 0;
    for (uint32_t j = j0, q = 0; j < j1; j++, q++) {
      ll[q] = S.lit[j];
      ml[q] = S.out[j];
      sl_ += ll[q];
      so_ += ll[q] + ml[q];
    }
    uint32_t tl, to;
    uint32_t pl = block_scan(S, sl_, &tl);
    uint32_t po = block_scan(S, so_, &to);
    bool bad = tl != nlit || to != blen;
    for (uint32_t j = j0, q = 0; j < j1; j++, q++) {
      S.lit[j] = (uint16_t)pl;
      S.out[j] = (uint16_t)po;
      const uint64_t of = (uint64_t)S.oflo[j] | ((uint64_t)S.ofhi[j] << 32);
      if (ml[q] == 0) bad |= (j != ns - 1) || of != 0;
      else bad |= ml[q] < A.m || of >= sb + po + ll[q];
      // matches with a source wholly in earlier blocks, listed in any order
      if (ml[q] && of + ml[q] <= sb) S.intl[atomicAdd(&S.nint, 1u)] = (uint16_t)j;
      pl += ll[q];
      po += ll[q] + ml[q];
    }
    if (t == 0) {
      S.lit[ns] = (uint16_t)min(tl, 65535u);
      S.out[ns] = (uint16_t)min(to, 65535u);
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return;
  }

  // ---- stage 3: literals straight to their tile positions; external matches
  {
    bool bad = false;
    // per-lane sequence cursor: literal i belongs to sequence j, the last one
    // with lit[j] <= i; its output position is i + (out[j] - lit[j])
    uint32_t j = 0, nxt = S.lit[1], dlt = S.out[0] - S.lit[0];
    auto seek = [&](uint32_t i) {              // binary search over lit[0..ns-1]
      uint32_t lo = 0, hi = ns ? ns - 1 : 0;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (S.lit[mid] <= i) lo = mid; else hi = mid - 1;
      }
      j = lo;
      nxt = S.lit[j + 1];
      dlt = (uint32_t)S.out[j] - (uint32_t)S.lit[j];
    };
    // called by every lane of the wave; lanes with act false store nothing
    auto place = [&](uint32_t i, uint32_t v, bool act) {
      if (__ballot(act && i >= nxt && j + 1 < ns)) {   // some lane entered a later sequence
        while (act && i >= nxt && j + 1 < ns) {
          j++;
          nxt = S.lit[j + 1];
          dlt = (uint32_t)S.out[j] - (uint32_t)S.lit[j];
        }
      }
      // i < lit[j+1] and the scans checked in stage 2 put i + dlt below
      // out[j+1] <= blen; the mask only keeps the store inside the tile
      if (act) S.tile[(i + dlt) & (kB - 1)] = (uint8_t)v;
    };
    if (sl.mode == kModeRans) {
      const uint32_t G = (sl.K + 63) >> 6, R = sl.n / sl.K, e = sl.n - R * sl.K;
      for (uint32_t g = wv; g < G; g += kWaves) {
        const uint32_t k = (g << 6) + lane;   // this lane's run starts at k*R + min(k, e)
        seek(min(k * R + min(k, e), sl.n - 1));
        if (!rans_lit(pay + sl.body, sl, g, A.P[kLit], S.lut, S.ring[wv], S.ringe[wv], place)) bad = true;
      }
    } else if (sl.mode == kModeRaw) {
      const uint8_t* src = pay + sl.body;
      for (uint32_t i0 = 0; i0 < sl.n; i0 += kWG) {
        const uint32_t i = i0 + t;
        place(i, i < sl.n ? src[i] : 0u, i < sl.n);
      }
    } else if (sl.mode == kModeConst) {
      for (uint32_t i0 = 0; i0 < sl.n; i0 += kWG) place(i0 + t, sl.csym, i0 + t < sl.n);
    }
    // matches with a source wholly in earlier blocks (listed in stage 2):
    // eight per wave at a time, one per 8-lane slot, each lane every eighth
    // byte, all loads in flight before the stores
    {
      const uint32_t nx = min(S.nint, ns), slot = lane >> 3, sub = lane & 7;
      for (uint32_t g0 = 8 * wv; g0 < nx; g0 += 8 * kWaves) {
        const uint32_t e = g0 + slot;
        const uint32_t q = e < nx ? min((uint32_t)S.intl[e], ns - 1) : 0u;
        const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
        const uint32_t M = e < nx ? (uint32_t)S.out[q + 1] - S.out[q] - L : 0u;
        const uint64_t of = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
        const uint32_t d0 = S.out[q] + L;
        for (uint32_t k0 = 0; k0 < M; k0 += 64) {
          uint32_t v[8];
          if (!A.addr) {                       // whole-file output: one base, byte offsets
            const uint8_t* p = A.out + of + k0 + sub;
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) v[u] = k0 + sub + 8 * u < M ? (uint32_t)p[8 * u] : 0u;
          } else {
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) {
              const uint32_t k = k0 + sub + 8 * u;
              v[u] = k < M ? src_byte(A, of + k, bad) : 0u;
            }
          }
#pragma unroll
          for (uint32_t u = 0; u < 8; u++) {
            const uint32_t k = k0 + sub + 8 * u;
            if (k < M && d0 + k < blen) S.tile[d0 + k] = (uint8_t)v[u];
          }
        }
      }
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return;
  }

  // ---- stage 4: matches whose source touches the block itself.
  // With period d = p - OF, out[p+k] = out[OF + (k mod d)] for every k (the
  // byte-sequential overlap rule unrolled); only the window OF..OF+min(d,M)-1
  // is read and it is final once every earlier match writing into it is done.
  // 4a: ordered list of these matches (ballot compaction, wave 0);
  // 4b: per match: destination, length, source (block-relative), period and
  //     the range of earlier such matches whose destinations its window
  //     meets (binary searches over the sorted destinations), packed into
  //     the sequence tables, which are no longer needed;
  // 4c: matches with an empty range copied by all waves in parallel;
  // 4d: the others copied by wave 0 in passes, each pass the matches whose
  //     earlier sources are complete.
  if (wv == 0) {
    uint32_t base = 0;
    for (uint32_t q0 = 0; q0 < ns; q0 += 64) {
      const uint32_t q = q0 + lane;
      bool in = false;
      if (q < ns) {
        const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
        const uint32_t M = (uint32_t)S.out[q + 1] - S.out[q] - L;
        const uint64_t of = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
        in = M && of + M > sb;
      }
      const uint64_t bal = __ballot(in);
      if (in) S.intl[base + mbcnt(bal)] = (uint16_t)q;
      base += (uint32_t)__popcll(bal);
    }
    if (lane == 0) S.nint = base;
  }
  __syncthreads();
  const uint32_t cnt = min(S.nint, ns);
  {
    // 4b phase 1: per match in registers (at most 5 per thread)
    uint32_t md0[5], mM[5], ms[5], md[5];
    const uint32_t per = (cnt + kWG - 1) / kWG, a0 = min(cnt, t * per), a1 = min(cnt, a0 + per);
    for (uint32_t a = a0, u = 0; a < a1; a++, u++) {
      const uint32_t q = min((uint32_t)S.intl[a], ns - 1);
      const uint32_t L = (uint32_t)S.lit[q + 1] - S.lit[q];
      const uint32_t M = min((uint32_t)S.out[q + 1] - S.out[q] - L, blen);
      const uint32_t d0 = S.out[q] + L;
      const uint64_t of = (uint64_t)S.oflo[q] | ((uint64_t)S.ofhi[q] << 32);
      const uint64_t dabs = sb + d0;
      md0[u] = d0;
      mM[u] = M;
      // of >= sb - M here (the source overlaps the block), so the relative
      // source fits in [-16384, 16384)
      ms[u] = (uint32_t)((int64_t)of - (int64_t)sb + 16384) & 0xFFFFu;
      md[u] = dabs > of ? (uint32_t)min<uint64_t>(dabs - of, 32767) : 1u;
    }
    __syncthreads();
    for (uint32_t a = a0, u = 0; a < a1; a++, u++) {
      S.lit[a] = (uint16_t)md0[u];
      S.out[a] = (uint16_t)mM[u];
    }
    __syncthreads();
    // 4b phase 2: the earlier matches whose destinations meet the window
    // form an index range [lo, hi) (destinations are sorted and disjoint);
    // the match is dependent if it is not empty.  The part of the range inside
    // the match's own 64-entry chunk is kept as bit positions (plo, phi).
    for (uint32_t a = a0, u = 0; a < a1; a++, u++) {
      const int32_t s = (int32_t)ms[u] - 16384;
      const uint32_t w = min(md[u], mM[u]);
      uint32_t lo = a, hi = a;
      if (s + (int32_t)w > 0) {
        const uint32_t ws = s > 0 ? (uint32_t)s : 0u, we = (uint32_t)(s + (int32_t)w);
        // two searches over [0, a) in lockstep: lo = first earlier match whose
        // destination ends after ws, hi = first whose destination starts at
        // or after we (hi >= lo: such a destination also ends after ws)
        uint32_t l1 = 0, h1 = a, l2 = 0, h2 = a;
        while (l1 < h1 || l2 < h2) {
          const uint32_t m1 = (l1 + h1) >> 1, m2 = (l2 + h2) >> 1;
          const uint32_t e1 = (uint32_t)S.lit[min(m1, a - 1)] + S.out[min(m1, a - 1)];
          const uint32_t b2 = S.lit[min(m2, a - 1)];
          if (l1 < h1) { if (e1 > ws) h1 = m1; else l1 = m1 + 1; }
          if (l2 < h2) { if (b2 >= we) h2 = m2; else l2 = m2 + 1; }
        }
        lo = l1;
        hi = l2;
      }
      const bool dep = lo < hi;
      const uint32_t c0 = a & ~63u;
      const uint32_t plo = max(lo, c0) - c0, phi = max(hi, c0) - c0;   // both <= 63
      S.intl[a] = (uint16_t)(plo | (phi << 8));
      S.oflo[a] = ms[u] | (md[u] << 16) | (dep ? 0x80000000u : 0u);
    }
  }
  __syncthreads();
  {
    bool bad = false;
    auto copy_match = [&](uint32_t a) {
      const uint32_t pk = S.oflo[a];
      const uint32_t d0 = S.lit[a], M = S.out[a];
      const int32_t s = (int32_t)(pk & 0xFFFFu) - 16384;
      const uint32_t d = (pk >> 16) & 0x7FFFu;
      if (d >= M) {                         // no overlap with itself: a plain copy
        for (uint32_t k = lane; k < M; k += 64) {
          if (d0 + k < blen) {
            const int32_t src = s + (int32_t)k;
            const uint32_t v = src >= 0 ? (uint32_t)S.tile[(uint32_t)src & (kB - 1)]
                                        : src_byte(A, sb + (int64_t)src, bad);
            S.tile[d0 + k] = (uint8_t)v;
          }
        }
        return;
      }
      // (c + lane) mod d, kept incrementally (a division only for d < 64)
      uint32_t r = d >= 64 ? lane : lane % d;
      const uint32_t r64 = d >= 64 ? 64u : 64u % d;
      for (uint32_t c = 0; c < M; c += 64) {
        const uint32_t k = c + lane;
        if (k < M && d0 + k < blen) {
          const int32_t src = s + (int32_t)r;
          const uint32_t v = src >= 0 ? (uint32_t)S.tile[(uint32_t)src & (kB - 1)]
                                      : src_byte(A, sb + (int64_t)src, bad);
          S.tile[d0 + k] = (uint8_t)v;
        }
        r += r64;
        if (r >= d) r -= d;
      }
    };
    // 4c: matches with an empty range, all waves: a wave tests 64 of its
    // entries (a = wv + 4 l) at once, then copies the ones that qualify
    for (uint32_t a0 = wv; a0 < cnt; a0 += kWaves * 64) {
      const uint32_t a = a0 + kWaves * lane;
      uint64_t m = __ballot(a < cnt && !(S.oflo[min(a, cnt - 1)] & 0x80000000u));
      while (m) {                              // wave-uniform
        const uint32_t l = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        copy_match(a0 + kWaves * l);
      }
    }
    __syncthreads();
    // 4d: dependent matches, wave 0, in passes over 64-entry chunks (every
    // earlier chunk is complete).  Lane l holds the predecessor bits of entry
    // c0 + l; a pass takes every pending match whose in-chunk predecessors
    // are all done, which includes the lowest pending one, so a chunk takes
    // at most 64 passes.  Matches of one pass do not read each other's
    // destinations.  The pass's matches are listed in LDS and copied eight at
    // a time, one per 8-lane slot, each lane every eighth byte (loads, then
    // stores); a match longer than 64 bytes or shorter than its period is
    // copied by the whole wave.  LDS operations of one wave are performed in
    // order, so a pass sees every earlier pass.
    if (wv == 0) {
      const uint32_t slot = lane >> 3, sub = lane & 7;
      for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
        const uint32_t a = c0 + lane;
        const bool have = a < cnt;
        const uint32_t rng = have ? (uint32_t)S.intl[a] : 0u;
        const uint32_t plo = rng & 63u, phi = (rng >> 8) & 63u;
        const uint64_t needm = phi > plo ? (1ull << phi) - (1ull << plo) : 0ull;
        const uint32_t mpk = have ? S.oflo[a] : 0u;
        const uint32_t mdl = have ? (uint32_t)S.lit[a] | ((uint32_t)S.out[a] << 16) : 0u;
        bool pending = have && (mpk & 0x80000000u);
        uint64_t done = ~__ballot(pending);
        for (uint32_t pass = 0; pass <= 64; pass++) {
          const bool ready = pending && (needm & ~done) == 0;
          const uint64_t m = __ballot(ready);
          if (!m) break;
          pending = pending && !ready;
          done |= m;
          if (ready) {                         // the pass's list, fields included
            const uint32_t pos = mbcnt(m);
            S.plist[pos] = (uint8_t)lane;
            S.ppk[pos] = mpk;
            S.pdl[pos] = mdl;
          }
          __builtin_amdgcn_wave_barrier();
          const uint32_t nr = (uint32_t)__popcll(m);
          for (uint32_t g0 = 0; g0 < nr; g0 += 8) {
            const uint32_t u = g0 + slot;
            const bool sv = u < nr;
            const uint32_t uu = sv ? u : 0u;
            const uint32_t j = c0 + (uint32_t)S.plist[uu];
            const uint32_t pkj = S.ppk[uu], dl = S.pdl[uu];
            const uint32_t dst = dl & 0xFFFFu, len = dl >> 16;
            const int32_t sj = (int32_t)(pkj & 0xFFFFu) - 16384;
            const uint32_t dj = (pkj >> 16) & 0x7FFFu;
            const bool simple = sv && dj >= len && len <= 64;
            uint32_t v[8];
            bool below = false;
#pragma unroll
            for (uint32_t q = 0; q < 8; q++) {
              const int32_t src = sj + (int32_t)(sub + 8 * q);
              v[q] = S.tile[(uint32_t)max(src, 0) & (kB - 1)];
              below |= simple && sub + 8 * q < len && src < 0;
            }
            if (__ballot(below)) {
#pragma unroll
              for (uint32_t q = 0; q < 8; q++) {
                const int32_t src = sj + (int32_t)(sub + 8 * q);
                if (simple && sub + 8 * q < len && src < 0) v[q] = src_byte(A, sb + (int64_t)src, bad);
              }
            }
#pragma unroll
            for (uint32_t q = 0; q < 8; q++) {
              const uint32_t k = sub + 8 * q;
              if (simple && k < len && dst + k < blen) S.tile[dst + k] = (uint8_t)v[q];
            }
            uint64_t slow = __ballot(sv && !simple && sub == 0);
            while (slow) {                     // wave-uniform
              const uint32_t l = (uint32_t)__builtin_ctzll(slow);
              slow &= slow - 1;
              copy_match((uint32_t)__builtin_amdgcn_readlane((int)j, (int)l));
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
        if (__ballot(pending)) bad = true;      // unreachable for a valid block
      }
    }
    if (bad) S.err = 1;
  }
  __syncthreads();
  if (S.err) {
    if (t == 0) latch(A.ctl, kStCorrupt);
    return;
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
}

// Once per workgroup: literal LUT image into LDS, small-stream cumulative tables.
__device__ void load_tables(Smem& S, const DevArgs& A) {
  const uint4* s = reinterpret_cast<const uint4*>(A.lut);
  uint4* d = reinterpret_cast<uint4*>(S.lut);
  for (uint32_t c = threadIdx.x; c < kLutLit / 4; c += kWG) d[c] = s[c];
  const uint32_t t = threadIdx.x;
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
  __syncthreads();
  // bucket index of each short stream: bucket b starts at slot b << bs
  for (uint32_t e = t; e < 3 * 256; e += kWG) {
    const uint32_t k = e >> 8, b = e & 255, P = A.P[1 + k];
    const uint32_t bs = P > 8 ? P - 8 : 0u;
    if ((b << bs) < (1u << P)) S.bkt[k][b] = (uint8_t)search_sym(S.cum[k], b << bs);
  }
}

__global__ void __launch_bounds__(kWG, 3) k_decode(DevArgs A) {   // 3 waves per SIMD: at most 168 VGPRs
  __shared__ Smem S;
  const uint32_t t = threadIdx.x;
  load_tables(S, A);
  __syncthreads();
  const uint32_t epoch = __hip_atomic_load(A.ctl + kCtlEpoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t qb = A.q_begin, qe = A.q_end;
  if (A.qptr) {
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
    // wait for every dependency's completion flag, then acquire
    const uint64_t d0 = ld64(A.arc + A.off_dep_ptr + 8ull * b);
    const uint64_t d1 = ld64(A.arc + A.off_dep_ptr + 8ull * (b + 1));
    for (uint64_t k = d0 + t; k < d1; k += kWG) {
      const uint32_t d = ld32(A.arc + A.off_dep_idx + 4 * k);
      uint32_t f;
      for (uint32_t spins = 0;
           (f = __hip_atomic_load(A.flags + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != epoch; spins++) {
        if (spins >= A.spin_limit) { watchdog(A.ctl, 1, b, d, f, epoch); break; }
        __builtin_amdgcn_s_sleep(1);
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

int lz_launch_decode_all(lz_handle* h, uint8_t* out, hipStream_t s) {
  DevArgs A = make_args(h);
  A.queue = h->ws.queue;
  A.out = out;
  const size_t smem = 0;   // all LDS is static
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
  const uint32_t g_wide = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (v.n_blocks + 255) / 256));
  hipLaunchKernelGGL(k_req_begin, dim3(1), dim3(256), 0, s, R);
  hipLaunchKernelGGL(k_req_spans, dim3(g_req), dim3(256), 0, s, R);
  hipLaunchKernelGGL(k_req_scan, dim3(1), dim3(1024), 0, s, R);
  hipLaunchKernelGGL(k_req_mark, dim3(g_wide), dim3(256), 0, s, R);
  hipLaunchKernelGGL(k_closure, dim3(std::min<uint32_t>(64, g_wide)), dim3(256), 0, s, R, spin);
  hipLaunchKernelGGL(k_req_levels, dim3(g_wide), dim3(256), 0, s, R);
  hipLaunchKernelGGL(k_req_level_scan, dim3(1), dim3(64), 0, s, R);
  hipLaunchKernelGGL(k_req_scatter, dim3(g_wide), dim3(256), 0, s, R);
  // decode the closure in level order (persistent, or one launch per level)
  DevArgs A = make_args(h);
  A.queue = h->ws.rqueue;
  A.qptr = h->ws.rlevel_ptr;
  A.addr = h->ws.addr;
  A.out = d_out;
  const uint32_t slots = (uint32_t)(h->n_cu * std::max(1u, h->tune.wg_per_cu));
  const uint32_t grid = (uint32_t)std::min<uint64_t>(slots, std::max<uint64_t>(1, v.n_blocks));
  if (h->tune.sync_mode == 1) {
    A.persistent = 1;
    A.q_begin = 0;
    A.q_end = 64;
    hipLaunchKernelGGL(k_decode, dim3(grid), dim3(kWG), 0, s, A);
  } else {
    for (uint32_t L = 0; L < v.n_levels; L++) {
      A.q_begin = L;
      A.q_end = L + 1;
      hipLaunchKernelGGL(k_decode, dim3(grid), dim3(kWG), 0, s, A);
    }
  }
  hipLaunchKernelGGL(k_req_gather, dim3(g_wide), dim3(256), 0, s, R);
  return launch_ok("request decode");
}
