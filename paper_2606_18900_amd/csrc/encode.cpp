// Host encoder (lz_encode) for container format v2.
//
// Global greedy match search whose matches carry absolute source positions in
// the decompressed output (paper, Background section), fixed-size blocks
// (Block Granularity section), four streams per block coded with interleaved
// rANS, dependency levels capped at max_level - 1, a read index for FASTQ
// (Read-Level Index subsection) and 64-bit positions (Scale section).
//
// Match policy at position p of block b (blocks [bB, min(bB+B, N))):
//   candidates: the hash chain of the first h bytes at p (most recent first,
//   at most C, none older than 2^R), then the first position ever seen with
//   that hash; length = common prefix of x[q:] and x[p:] capped at the block
//   end; level lv = 0 for a source inside the block, else 1 + the highest level
//   among the earlier blocks the source touches; score = length - beta * lv;
//   drop lv > D - 1 or score < m; best score wins, then lower lv, then the
//   first candidate seen.  A match advances p by its length, otherwise p += 1.
// Levels feed back into later choices, so the policy is sequential; parse_impl
// computes exactly those choices with host threads (see there), and the
// per-block stream coding runs on host threads too.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <new>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <memory>
#include <vector>

#include "lz.h"
#include "lz_internal.h"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t load_le(const uint8_t* p, uint32_t n) {
  uint64_t v = 0;
  std::memcpy(&v, p, n);  // little-endian host
  return v;
}

struct Hasher {
  uint32_t h, H;
  uint64_t mask0, mask1;
  Hasher(uint32_t h_, uint32_t H_) : h(h_), H(H_) {
    uint32_t n0 = h < 8 ? h : 8, n1 = h > 8 ? h - 8 : 0;
    mask0 = n0 == 8 ? ~0ull : ((1ull << (8 * n0)) - 1);
    mask1 = n1 == 8 ? ~0ull : ((1ull << (8 * n1)) - 1);
  }
  // requires p + h <= n; reads exactly h bytes unless 16 are available
  inline uint64_t operator()(const uint8_t* x, uint64_t p, uint64_t n) const { return mix(x, p, n) >> (64 - H); }
  // the 64-bit value whose top H bits are the hash
  inline uint64_t mix(const uint8_t* x, uint64_t p, uint64_t n) const {
    uint64_t v0, v1;
    if (p + 16 <= n) {
      std::memcpy(&v0, x + p, 8);
      std::memcpy(&v1, x + p + 8, 8);
      v0 &= mask0;
      v1 &= mask1;
    } else {
      v0 = load_le(x + p, h < 8 ? h : 8);
      v1 = h > 8 ? load_le(x + p + 8, h - 8) : 0;
    }
    uint64_t t = v0 * kGolden;
    t = (t << 29) | (t >> 35);
    return (t ^ v1) * kGolden;
  }
};

inline uint64_t lcp(const uint8_t* x, uint64_t q, uint64_t p, uint64_t cap) {
  uint64_t L = 0;
  while (L + 8 <= cap) {
    uint64_t a, b;
    std::memcpy(&a, x + q + L, 8);
    std::memcpy(&b, x + p + L, 8);
    uint64_t d = a ^ b;
    if (d) return L + (__builtin_ctzll(d) >> 3);
    L += 8;
  }
  while (L < cap && x[q + L] == x[p + L]) L++;
  return L;
}

struct Parse {
  std::vector<uint32_t> ll, ml;
  std::vector<uint64_t> of;
  std::vector<uint64_t> seq_ptr;   // n_blocks + 1
  std::vector<uint16_t> level;
  std::vector<uint64_t> dep_ptr;   // n_blocks + 1
  std::vector<uint32_t> dep_idx;
};

template <typename F>
void parallel_for(uint64_t n, unsigned threads, F&& f);

// The parse is defined sequentially (see the file comment); this computes the
// same sequences with host threads:
//  1. the hash of every insertable position;
//  2. for every position its previous same-hash position and, per hash, the
//     first position — built per hash partition, each partition scanned in
//     increasing position order with a cache-sized local head table.  Walking
//     these links from p visits exactly what the sequential chain holds at p;
//  3. blocks are claimed in increasing order; a block's parse only needs the
//     final level of an earlier block when a candidate from it could still be
//     accepted (length - beta >= m), and then waits for that block to finish.
//     Earlier blocks are claimed earlier, so every wait ends.
template <typename Pos>
int parse_impl(const uint8_t* x, uint64_t n, const lz_params& pr, unsigned threads, Parse& out) {
  const uint32_t bl = pr.block_log2;
  const uint64_t B = 1ull << bl, nb = (n + B - 1) >> bl;
  const uint32_t h = pr.hash_len, m = pr.min_match, D = pr.max_level, H = pr.hash_bits;
  const uint64_t C = pr.chain_depth ? pr.chain_depth : ~0ull;
  const uint64_t win = pr.window_log2 ? (1ull << pr.window_log2) : ~0ull;
  const int64_t beta = pr.level_penalty;
  const Pos kNone = (Pos)~(Pos)0;
  const Hasher hash(h, H);
  const uint64_t nh = n >= h ? n - h + 1 : 0;
  const uint64_t chunk = 1 << 20, nchunks = (nh + chunk - 1) / chunk;
  std::vector<uint32_t> hv(nh ? nh : 1);
  parallel_for(nchunks, threads, [&](uint64_t c, unsigned) {
    const uint64_t e = std::min(nh, (c + 1) * chunk);
    for (uint64_t p = c * chunk; p < e; p++) hv[p] = (uint32_t)hash(x, p, n);
  });
  // 2. counting sort of positions by hash partition (top bits), then links
  const uint32_t pbits = std::min<uint32_t>(8, H), np = 1u << pbits, shift = H - pbits;
  std::vector<uint64_t> cnt(nchunks * np, 0), pstart(np + 1, 0);
  parallel_for(nchunks, threads, [&](uint64_t c, unsigned) {
    const uint64_t e = std::min(nh, (c + 1) * chunk);
    uint64_t* hc = &cnt[c * np];
    for (uint64_t p = c * chunk; p < e; p++) hc[hv[p] >> shift]++;
  });
  for (uint32_t k = 0; k < np; k++) {
    uint64_t tot = 0;
    for (uint64_t c = 0; c < nchunks; c++) { uint64_t v = cnt[c * np + k]; cnt[c * np + k] = tot; tot += v; }
    pstart[k + 1] = pstart[k] + tot;
  }
  std::vector<Pos> order(nh ? nh : 1);
  parallel_for(nchunks, threads, [&](uint64_t c, unsigned) {
    const uint64_t e = std::min(nh, (c + 1) * chunk);
    std::vector<uint64_t> cur(np);
    for (uint32_t k = 0; k < np; k++) cur[k] = pstart[k] + cnt[c * np + k];
    for (uint64_t p = c * chunk; p < e; p++) order[cur[hv[p] >> shift]++] = (Pos)p;
  });
  std::vector<Pos> prev(nh ? nh : 1), first(1ull << H, kNone);
  parallel_for(np, threads, [&](uint64_t k, unsigned) {
    std::vector<Pos> head(1ull << shift, kNone);
    const uint32_t lmask = (1u << shift) - 1;
    for (uint64_t i = pstart[k]; i < pstart[k + 1]; i++) {
      const Pos p = order[i];
      const uint32_t hh = hv[p];
      prev[p] = head[hh & lmask];
      head[hh & lmask] = p;
      if (first[hh] == kNone) first[hh] = p;
    }
  });
  std::vector<Pos>().swap(order);

  // 3. greedy parse of the blocks on worker threads
  struct BlockOut {
    std::vector<uint32_t> ll, ml, deps;
    std::vector<uint64_t> of;
  };
  std::vector<BlockOut> bo(nb);
  out.level.assign(nb, 0);
  std::unique_ptr<std::atomic<uint8_t>[]> done(new std::atomic<uint8_t>[nb ? nb : 1]);
  for (uint64_t b = 0; b < nb; b++) done[b].store(0, std::memory_order_relaxed);
  std::atomic<uint64_t> next{0};
  auto level_of = [&](uint64_t k) -> uint32_t {
    while (!done[k].load(std::memory_order_acquire)) std::this_thread::yield();
    return out.level[k];
  };
  auto work = [&]() {
    for (;;) {
      const uint64_t b = next.fetch_add(1);
      if (b >= nb) break;
      BlockOut& o = bo[b];
      const uint64_t sb = b << bl, eb = std::min(sb + B, n);
      uint64_t p = sb, lit = sb;
      uint32_t blevel = 0;
      while (p < eb) {
        uint64_t bestL = 0, bestQ = 0;
        uint32_t bestLv = 0;
        int64_t bestSc = 0;
        if (p + m <= eb) {
          Pos a = first[hv[p]];
          if ((uint64_t)a >= p) a = kNone;     // no earlier position with this hash
          bool anchor_seen = false;
          auto consider = [&](uint64_t q) {
            const uint64_t L = lcp(x, q, p, eb - p);
            if (L < m) return;
            uint32_t lv = 0;
            if (q < sb) {
              // best case for a source in earlier blocks is level 1: if even
              // that loses (or is rejected), the candidate cannot change the
              // choice, so its level is not needed
              const int64_t ub = (int64_t)L - beta;
              if (ub < (int64_t)m) return;
              if (bestL && (ub < bestSc || (ub == bestSc && bestLv <= 1))) return;
              const uint64_t hi = std::min(q + L, sb);
              uint32_t mx = 0;
              for (uint64_t k = q >> bl; k <= (hi - 1) >> bl; k++) mx = std::max(mx, level_of(k));
              lv = mx + 1;
            }
            if (lv > D - 1) return;
            const int64_t sc = (int64_t)L - beta * (int64_t)lv;
            if (sc < (int64_t)m) return;
            if (bestL == 0 || sc > bestSc || (sc == bestSc && lv < bestLv)) {
              bestSc = sc;
              bestL = L;
              bestQ = q;
              bestLv = lv;
            }
          };
          Pos q = prev[p];
          uint64_t c = 0;
          while (q != kNone && c < C && p - (uint64_t)q <= win) {
            if (q == a) anchor_seen = true;
            consider(q);
            q = prev[q];
            c++;
          }
          if (a != kNone && !anchor_seen) consider(a);
        }
        if (bestL) {
          o.ll.push_back((uint32_t)(p - lit));
          o.ml.push_back((uint32_t)bestL);
          o.of.push_back(bestQ);
          if (bestQ < sb) {
            const uint64_t hi = std::min(bestQ + bestL, sb);
            for (uint64_t k = bestQ >> bl; k <= (hi - 1) >> bl; k++) o.deps.push_back((uint32_t)k);
          }
          blevel = std::max(blevel, bestLv);
          p += bestL;
          lit = p;
        } else {
          p++;
        }
      }
      if (lit < eb) {
        o.ll.push_back((uint32_t)(eb - lit));
        o.ml.push_back(0);
        o.of.push_back(0);
      }
      std::sort(o.deps.begin(), o.deps.end());
      o.deps.erase(std::unique(o.deps.begin(), o.deps.end()), o.deps.end());
      out.level[b] = (uint16_t)blevel;
      done[b].store(1, std::memory_order_release);
    }
  };
  {
    std::vector<std::thread> ts;
    for (unsigned t = 1; t < threads; t++) ts.emplace_back(work);
    work();
    for (auto& t : ts) t.join();
  }
  out.seq_ptr.assign(nb + 1, 0);
  out.dep_ptr.assign(nb + 1, 0);
  for (uint64_t b = 0; b < nb; b++) {
    out.seq_ptr[b + 1] = out.seq_ptr[b] + bo[b].ll.size();
    out.dep_ptr[b + 1] = out.dep_ptr[b] + bo[b].deps.size();
  }
  out.ll.resize(out.seq_ptr[nb]);
  out.ml.resize(out.seq_ptr[nb]);
  out.of.resize(out.seq_ptr[nb]);
  out.dep_idx.resize(out.dep_ptr[nb]);
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    std::copy(bo[b].ll.begin(), bo[b].ll.end(), out.ll.begin() + out.seq_ptr[b]);
    std::copy(bo[b].ml.begin(), bo[b].ml.end(), out.ml.begin() + out.seq_ptr[b]);
    std::copy(bo[b].of.begin(), bo[b].of.end(), out.of.begin() + out.seq_ptr[b]);
    std::copy(bo[b].deps.begin(), bo[b].deps.end(), out.dep_idx.begin() + out.dep_ptr[b]);
  });
  return LZ_OK;
}

// Segmented parse (segment_log2 > 0), for inputs too large for the global
// parse's per-position tables.  Segments of S = 2^segment_log2 bytes (whole
// blocks) are taken in order by host threads.  Segment s looks for sources in
//   (a) its own earlier positions whose hash has the same low 18 bits and
//       the same 8 bits above them: the min(C, 4) most recent ones (a 4-way
//       bucket of 24-bit segment positions with the 8 bits beside them, most
//       recent first), none older than 2^window_log2 when set;
//   (b) per hash, the first position ever seen, when it lies in a segment
//       s - kSegLag or earlier.  The table entry also keeps 24 further bits of
//       that position's hash, so a position whose hash only shares the top
//       bits is not read.
// Before segment s starts, every segment up to s - kSegLag is complete, so
// (b) finds the same position whatever the threads' timing, and every level
// the scoring needs is final: the archive depends only on the input and the
// parameters.  Scoring, tie-breaking and the level cap are those of the
// global parse.  Hashes are computed a block ahead and the table lines of
// position p + kAhead are prefetched while p is parsed.
constexpr uint64_t kSegLag = 32;
constexpr uint32_t kWays = 4;
constexpr uint64_t kAhead = 32;

int parse_segmented(const uint8_t* x, uint64_t n, const lz_params& pr, unsigned threads, Parse& out) {
  const uint32_t bl = pr.block_log2;
  const uint64_t B = 1ull << bl, nb = (n + B - 1) >> bl;
  const uint32_t h = pr.hash_len, m = pr.min_match, D = pr.max_level;
  const uint32_t H = std::min<uint32_t>(pr.hash_bits, 28);
  const uint32_t HL = 18;                                   // per-segment buckets
  const uint64_t C = std::min<uint64_t>(pr.chain_depth ? pr.chain_depth : kWays, kWays);
  const uint64_t win = pr.window_log2 ? (1ull << pr.window_log2) : ~0ull;
  const int64_t beta = pr.level_penalty;
  const uint32_t sl = pr.segment_log2;
  const uint64_t S = 1ull << sl, nseg = (n + S - 1) >> sl;
  const Hasher hash(h, H);
  // first-seen entries: 24 tag bits << 40 | position (positions below 2^40)
  constexpr uint64_t kNone = ~0ull, kPosMask = (1ull << 40) - 1;
  if (n >= kPosMask) return LZ_EINVAL;
  std::unique_ptr<std::atomic<uint64_t>[]> first(new (std::nothrow) std::atomic<uint64_t>[1ull << H]);
  if (!first) return LZ_EINVAL;
  parallel_for(1ull << (H > 20 ? H - 20 : 0), threads, [&](uint64_t c, unsigned) {
    const uint64_t lo = c << 20, hi = std::min<uint64_t>(1ull << H, lo + (1ull << 20));
    for (uint64_t i = lo; i < hi; i++) first[i].store(kNone, std::memory_order_relaxed);
  });
  auto tag_of = [&](uint64_t mx) -> uint64_t { return ((mx >> (40 - H)) & 0xFFFFFFull) << 40; };
  struct BlockOut {
    std::vector<uint32_t> ll, ml, deps;
    std::vector<uint64_t> of;
  };
  std::vector<BlockOut> bo(nb);
  out.level.assign(nb, 0);
  std::unique_ptr<std::atomic<uint8_t>[]> seg_done(new std::atomic<uint8_t>[nseg ? nseg : 1]);
  for (uint64_t i = 0; i < nseg; i++) seg_done[i].store(0, std::memory_order_relaxed);
  std::atomic<uint64_t> next{0}, low{0};     // low: every segment below it is complete
  std::mutex mu;
  auto finish = [&](uint64_t sg) {
    seg_done[sg].store(1, std::memory_order_release);
    std::lock_guard<std::mutex> g(mu);
    uint64_t w = low.load(std::memory_order_relaxed);
    while (w < nseg && seg_done[w].load(std::memory_order_acquire)) w++;
    low.store(w, std::memory_order_release);
  };
  auto work = [&]() {
    // bucket k: entries [kWays k, kWays k + kWays): 8 tag bits << 24 |
    // (position - s0 + 1); 0 = empty
    std::vector<uint32_t> bkt((size_t)kWays << HL);
    std::vector<uint64_t> hv(B + kAhead);
    const uint64_t lmask = (1ull << HL) - 1;
    for (;;) {
      const uint64_t sg = next.fetch_add(1);
      if (sg >= nseg) break;
      const uint64_t need = sg >= kSegLag ? sg - kSegLag + 1 : 0;
      while (low.load(std::memory_order_acquire) < need) std::this_thread::sleep_for(std::chrono::microseconds(50));
      const uint64_t s0 = sg << sl, s1 = std::min(n, s0 + S);
      const uint64_t far = need << sl;           // first-seen sources must lie below this
      std::fill(bkt.begin(), bkt.end(), 0u);
      const uint64_t nh = n >= h ? n - h + 1 : 0;   // positions with a hash
      uint64_t ins = s0;                             // next position to insert
      for (uint64_t b = s0 >> bl; b << bl < s1; b++) {
        BlockOut& o = bo[b];
        const uint64_t sb = b << bl, eb = std::min(sb + B, n);
        // hashes of [sb, eb + kAhead) within the segment
        const uint64_t he = std::min({eb + kAhead, s1, nh});
        for (uint64_t q = sb; q < he; q++) hv[q - sb] = hash.mix(x, q, n);
        auto hash_at = [&](uint64_t q) -> uint64_t { return hv[q - sb] >> (64 - H); };
        // bucket of the low 18 bits of the 64-bit mix, tag of the 8 above
        auto bucket_at = [&](uint64_t q) -> uint64_t { return hv[q - sb] & lmask; };
        auto btag_at = [&](uint64_t q) -> uint32_t { return (uint32_t)((hv[q - sb] >> HL) & 0xFFu) << 24; };
        auto prefetch = [&](uint64_t q) {
          if (q < he) {
            __builtin_prefetch(&bkt[bucket_at(q) * kWays], 1);
            __builtin_prefetch(&first[hash_at(q)], 1);
          }
        };
        auto insert_to = [&](uint64_t e) {
          for (; ins < e && ins < nh; ins++) {
            prefetch(ins + kAhead);
            const uint64_t hq = hash_at(ins);
            uint32_t* bk = &bkt[bucket_at(ins) * kWays];
            for (uint32_t w = kWays - 1; w; w--) bk[w] = bk[w - 1];
            bk[0] = btag_at(ins) | (uint32_t)(ins - s0 + 1);
            std::atomic<uint64_t>& f = first[hq];
            const uint64_t mine = tag_of(hv[ins - sb]) | ins;
            uint64_t cur = f.load(std::memory_order_relaxed);
            while ((cur & kPosMask) > ins && !f.compare_exchange_weak(cur, mine, std::memory_order_relaxed)) {
            }
          }
          if (ins < e) ins = e;
        };
        uint64_t p = sb, lit = sb;
        uint32_t blevel = 0;
        while (p < eb) {
          insert_to(p);
          prefetch(p + kAhead);
          uint64_t bestL = 0, bestQ = 0;
          uint32_t bestLv = 0;
          int64_t bestSc = 0;
          if (p + m <= eb) {
            const uint64_t hp = hash_at(p);
            auto consider = [&](uint64_t q) {
              const uint64_t L = lcp(x, q, p, eb - p);
              if (L < m) return;
              uint32_t lv = 0;
              if (q < sb) {
                const uint64_t hi = std::min(q + L, sb);
                uint32_t mx = 0;
                for (uint64_t k = q >> bl; k <= (hi - 1) >> bl; k++) mx = std::max<uint32_t>(mx, out.level[k]);
                lv = mx + 1;
              }
              if (lv > D - 1) return;
              const int64_t sc = (int64_t)L - beta * (int64_t)lv;
              if (sc < (int64_t)m) return;
              if (bestL == 0 || sc > bestSc || (sc == bestSc && lv < bestLv)) {
                bestSc = sc;
                bestL = L;
                bestQ = q;
                bestLv = lv;
              }
            };
            // (a) own segment, most recent first
            const uint32_t* bk = &bkt[bucket_at(p) * kWays];
            const uint32_t tg = btag_at(p);
            for (uint64_t c = 0; c < C && bk[c]; c++) {
              const uint64_t q = s0 + (bk[c] & 0xFFFFFFu) - 1;
              if (p - q > win) break;
              if ((bk[c] & 0xFF000000u) == tg) consider(q);
            }
            // (b) first position seen with this hash, kSegLag or more segments back
            const uint64_t fa = first[hp].load(std::memory_order_relaxed);
            const uint64_t a = fa & kPosMask;
            if (fa != kNone && (fa & ~kPosMask) == tag_of(hv[p - sb]) && a < far) consider(a);
          }
          if (bestL) {
            o.ll.push_back((uint32_t)(p - lit));
            o.ml.push_back((uint32_t)bestL);
            o.of.push_back(bestQ);
            if (bestQ < sb) {
              const uint64_t hi = std::min(bestQ + bestL, sb);
              for (uint64_t k = bestQ >> bl; k <= (hi - 1) >> bl; k++) o.deps.push_back((uint32_t)k);
            }
            blevel = std::max(blevel, bestLv);
            p += bestL;
            lit = p;
          } else {
            p++;
          }
        }
        insert_to(eb);
        if (lit < eb) {
          o.ll.push_back((uint32_t)(eb - lit));
          o.ml.push_back(0);
          o.of.push_back(0);
        }
        std::sort(o.deps.begin(), o.deps.end());
        o.deps.erase(std::unique(o.deps.begin(), o.deps.end()), o.deps.end());
        out.level[b] = (uint16_t)blevel;
      }
      finish(sg);
    }
  };
  {
    std::vector<std::thread> ts;
    for (unsigned t = 1; t < threads; t++) ts.emplace_back(work);
    work();
    for (auto& t : ts) t.join();
  }
  out.seq_ptr.assign(nb + 1, 0);
  out.dep_ptr.assign(nb + 1, 0);
  for (uint64_t b = 0; b < nb; b++) {
    out.seq_ptr[b + 1] = out.seq_ptr[b] + bo[b].ll.size();
    out.dep_ptr[b + 1] = out.dep_ptr[b] + bo[b].deps.size();
  }
  out.ll.resize(out.seq_ptr[nb]);
  out.ml.resize(out.seq_ptr[nb]);
  out.of.resize(out.seq_ptr[nb]);
  out.dep_idx.resize(out.dep_ptr[nb]);
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    std::copy(bo[b].ll.begin(), bo[b].ll.end(), out.ll.begin() + out.seq_ptr[b]);
    std::copy(bo[b].ml.begin(), bo[b].ml.end(), out.ml.begin() + out.seq_ptr[b]);
    std::copy(bo[b].of.begin(), bo[b].of.end(), out.of.begin() + out.seq_ptr[b]);
    std::copy(bo[b].deps.begin(), bo[b].deps.end(), out.dep_idx.begin() + out.dep_ptr[b]);
    bo[b] = BlockOut();
  });
  return LZ_OK;
}

// ---------------------------------------------------------------- rANS
// Normalise counts to sum 2^P (floor(c*M/T), at least 1 per seen symbol;
// remainder to the most frequent symbol, lowest value on ties; an excess is
// removed one unit at a time from the largest f > 1, lowest value on ties).
int normalize(const uint64_t* counts, uint32_t P, uint16_t* freq) {
  uint64_t T = 0;
  for (int s = 0; s < 256; s++) T += counts[s];
  std::memset(freq, 0, 512);
  if (!T) return LZ_OK;
  const uint64_t M = 1ull << P;
  int64_t sum = 0;
  for (int s = 0; s < 256; s++)
    if (counts[s]) {
      uint64_t f = std::max<uint64_t>(1, counts[s] * M / T);
      freq[s] = (uint16_t)f;
      sum += (int64_t)f;
    }
  int64_t d = (int64_t)M - sum;
  if (d > 0) {
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (counts[s] && (best < 0 || counts[s] > counts[best])) best = s;
    freq[best] = (uint16_t)(freq[best] + d);
  }
  while (d < 0) {
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (freq[s] > 1 && (best < 0 || freq[s] > freq[best])) best = s;
    if (best < 0) return LZ_EINVAL;
    freq[best]--;
    d++;
  }
  return LZ_OK;
}

// largest power of two <= n / per_lane, at least 1, at most max_lanes
// (16 symbols per lane for literals, 4 for the short CMD/MLEN/OFF streams)
uint32_t lanes_for(uint32_t n, uint32_t max_lanes, uint32_t per_lane) {
  uint32_t q = n / per_lane, k = 1;
  while (k * 2 <= q) k *= 2;
  return std::min(k, max_lanes);
}

struct Table {
  uint16_t f[256];
  uint32_t c[257];
  uint32_t P;
};

// Encode sym[0..n) with K lanes.  Lane k owns the run of n/K consecutive
// symbols (one more for the first n mod K lanes) that the decoder takes one per
// round; decode slot o = r*K + k is round r of lane k.  The encoder walks the
// slots backwards and stores each group's words in slot order.
void rans_body(const uint8_t* sym, uint32_t n, const Table& t, uint32_t K,
               std::vector<uint8_t>& body, uint32_t& n_words) {
  const uint32_t G = (K + 63) / 64, R = n / K, e = n % K;
  const uint64_t slots = (uint64_t)((n + K - 1) / K) * K;
  uint32_t x[256];
  uint64_t start[257];
  for (uint32_t k = 0; k < K; k++) {
    x[k] = 1u << 16;
    start[k] = (uint64_t)k * R + std::min(k, e);
  }
  std::vector<uint16_t> w(slots);
  std::vector<uint8_t> has(slots, 0);
  for (uint64_t o = slots; o-- > 0;) {
    const uint32_t r = (uint32_t)(o / K), k = (uint32_t)(o % K);
    if (r >= R + (k < e ? 1u : 0u)) continue;
    const uint32_t s = sym[start[k] + r], f = t.f[s];
    uint64_t xm = (uint64_t)f << (32 - t.P);
    uint64_t v = x[k];
    if (v >= xm) {
      w[o] = (uint16_t)(v & 0xFFFF);
      has[o] = 1;
      v >>= 16;
    }
    x[k] = (uint32_t)((v / f) * (1ull << t.P) + (v % f) + t.c[s]);
  }
  uint32_t gw[4] = {0, 0, 0, 0}, nw = 0;
  for (uint64_t o = 0; o < slots; o++)
    if (has[o]) { gw[(o % K) >> 6]++; nw++; }
  body.resize(4ull * K + 4ull * G + 2ull * nw);
  uint8_t* op = body.data();
  for (uint32_t k = 0; k < K; k++, op += 4) std::memcpy(op, &x[k], 4);
  for (uint32_t g = 0; g < G; g++, op += 4) std::memcpy(op, &gw[g], 4);
  // words of group g in slot order: lanes 64g..64g+63 of each round
  for (uint32_t g = 0; g < G; g++) {
    const uint32_t k0 = 64 * g, k1 = std::min(K, k0 + 64);
    for (uint64_t r0 = 0; r0 < slots; r0 += K)
      for (uint32_t k = k0; k < k1; k++)
        if (has[r0 + k]) { std::memcpy(op, &w[r0 + k], 2); op += 2; }
  }
  n_words = nw;
}

void put_stream(std::vector<uint8_t>& outb, const uint8_t* sym, uint32_t n, const Table& t,
                uint32_t max_lanes, uint32_t per_lane) {
  uint8_t hdr[16] = {0};
  std::memcpy(hdr + 4, &n, 4);
  auto pad = [&]() { while (outb.size() & 15) outb.push_back(0); };
  if (n == 0) {
    hdr[0] = kModeEmpty;
    outb.insert(outb.end(), hdr, hdr + 16);
    return;
  }
  bool same = true;
  for (uint32_t i = 1; i < n && same; i++) same = sym[i] == sym[0];
  if (same) {
    hdr[0] = kModeConst;
    hdr[1] = sym[0];
    outb.insert(outb.end(), hdr, hdr + 16);
    return;
  }
  uint32_t K = lanes_for(n, max_lanes, per_lane), nw = 0;
  std::vector<uint8_t> body;
  rans_body(sym, n, t, K, body, nw);
  if (body.size() >= n) {
    hdr[0] = kModeRaw;
    std::memcpy(hdr + 12, &n, 4);
    outb.insert(outb.end(), hdr, hdr + 16);
    outb.insert(outb.end(), sym, sym + n);
  } else {
    hdr[0] = kModeRans;
    uint16_t k16 = (uint16_t)K;
    uint32_t bl = (uint32_t)body.size();
    std::memcpy(hdr + 2, &k16, 2);
    std::memcpy(hdr + 8, &nw, 4);
    std::memcpy(hdr + 12, &bl, 4);
    outb.insert(outb.end(), hdr, hdr + 16);
    outb.insert(outb.end(), body.begin(), body.end());
  }
  pad();
}

uint64_t fnv1a(const uint8_t* p, uint64_t n, uint64_t h) {
  for (uint64_t i = 0; i < n; i++) h = (h ^ p[i]) * kFnvPrime;
  return h;
}

template <typename F>
void parallel_for(uint64_t n, unsigned threads, F&& f) {
  if (threads <= 1 || n < 2) {
    for (uint64_t i = 0; i < n; i++) f(i, 0u);
    return;
  }
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> ts;
  for (unsigned t = 0; t < threads; t++)
    ts.emplace_back([&, t]() {
      for (;;) {
        uint64_t i = next.fetch_add(1);
        if (i >= n) break;
        f(i, t);
      }
    });
  for (auto& t : ts) t.join();
}

// Source rebasing, an encoder choice the format leaves free: a match that
// does not overlap itself and whose source window lies wholly inside the
// destination of an earlier match of its block (one not overlapping itself,
// so that destination equals its source byte for byte) reads from that
// match's source instead; repeated until no match holds the window (each
// step goes to a match of smaller index).  Matches are taken in sequence
// order, so earlier sources are final.  The window moves into bytes the block
// already depends on: dependencies and levels stay; in-block copy chains, and
// the decoder's dependency passes, get shorter.  Blocks are independent.
void rebase_sources(Parse& ps, uint64_t nb, uint32_t bl, unsigned threads) {
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    const uint64_t s0 = ps.seq_ptr[b], s1 = ps.seq_ptr[b + 1];
    std::vector<uint64_t> dst, idx;             // the block's matches: destination, sequence index
    uint64_t pos = b << bl;
    for (uint64_t q = s0; q < s1; q++) {
      pos += ps.ll[q];
      if (ps.ml[q]) { dst.push_back(pos); idx.push_back(q); }
      pos += ps.ml[q];
    }
    for (uint64_t m = 0; m < dst.size(); m++) {
      const uint64_t q = idx[m], p = dst[m], M = ps.ml[q];
      for (;;) {
        const uint64_t o = ps.of[q];
        if (p - o < M) break;                                    // overlaps itself
        // the last earlier match whose destination starts at or before o
        const uint64_t c1 = (uint64_t)(std::upper_bound(dst.begin(), dst.begin() + m, o) - dst.begin());
        if (!c1) break;
        const uint64_t c = c1 - 1, qc = idx[c], pc = dst[c], Mc = ps.ml[qc], oc = ps.of[qc];
        if (o + M > pc + Mc || pc - oc < Mc) break;              // not inside, or it overlaps itself
        ps.of[q] = oc + (o - pc);
      }
    }
  });
}

int check(const lz_params& p) {
  if (p.block_log2 < 6 || p.block_log2 > 15) return LZ_EINVAL;
  if (p.max_level < 1 || p.max_level > 64) return LZ_EINVAL;
  if (p.hash_len < 4 || p.hash_len > 16) return LZ_EINVAL;
  if (p.min_match < p.hash_len || p.min_match > 255) return LZ_EINVAL;
  if (p.hash_bits < 8 || p.hash_bits > 30) return LZ_EINVAL;
  if (p.window_log2 > 40 || p.chain_depth > 65535) return LZ_EINVAL;
  if (p.lit_lanes < 1 || p.lit_lanes > 256 || p.seq_lanes < 1 || p.seq_lanes > 64) return LZ_EINVAL;
  for (int k = 0; k < 4; k++)
    if (p.prob_bits[k] < 8 || p.prob_bits[k] > 12) return LZ_EINVAL;
  if (p.kind > 2 || p.level_penalty > 255) return LZ_EINVAL;
  if (p.segment_log2 && (p.segment_log2 < p.block_log2 || p.segment_log2 > 24)) return LZ_EINVAL;
  return LZ_OK;
}

}  // namespace

extern "C" int lz_params_default(lz_params* p) {
  if (!p) return lz_fail(LZ_EINVAL, "lz_params_default: null");
  p->block_log2 = 14;
  p->max_level = 64;
  p->min_match = 16;
  p->hash_len = 16;
  p->hash_bits = 20;
  p->chain_depth = 64;
  p->window_log2 = 0;
  p->lit_lanes = 256;
  p->seq_lanes = 64;
  p->prob_bits[0] = 12;
  p->prob_bits[1] = p->prob_bits[2] = p->prob_bits[3] = 10;
  p->kind = 0;
  p->level_penalty = 32;
  p->threads = 0;
  p->segment_log2 = 0;
  return LZ_OK;
}

extern "C" void lz_free(void* p) { std::free(p); }

extern "C" int lz_encode(const uint8_t* x, uint64_t n, const lz_params* pp, uint8_t** archive,
                         uint64_t* archive_len) {
  if (!pp || !archive || !archive_len || (n && !x)) return lz_fail(LZ_EINVAL, "lz_encode: null argument");
  const lz_params pr = *pp;
  if (check(pr)) return lz_fail(LZ_EINVAL, "lz_encode: parameter out of range");
  unsigned threads = pr.threads ? pr.threads : std::max(1u, std::thread::hardware_concurrency());
  const uint32_t bl = pr.block_log2;
  const uint64_t B = 1ull << bl, nb = (n + B - 1) >> bl;
  uint32_t w = 1;
  {
    uint64_t v = n ? n - 1 : 0;
    uint32_t bits = 0;
    while (v) { bits++; v >>= 1; }
    w = std::max(1u, (bits + 7) / 8);
  }
  // read index: start of line 4r, counted by newlines
  std::vector<uint64_t> ridx;
  uint32_t max_rec = 0;
  if (pr.kind == 1) {
    if (n && x[n - 1] != '\n') return lz_fail(LZ_EINVAL, "lz_encode: FASTQ input does not end in a newline");
    ridx.push_back(0);
    uint64_t line = 0;
    for (const uint8_t* q = x; (q = (const uint8_t*)std::memchr(q, '\n', (size_t)(x + n - q)));) {
      q++;
      if (++line % 4 == 0) ridx.push_back((uint64_t)(q - x));
      if (q >= x + n) break;
    }
    if (line % 4) return lz_fail(LZ_EINVAL, "lz_encode: FASTQ input is not whole 4-line records");
    for (size_t r = 0; r + 1 < ridx.size(); r++) {
      uint64_t len = ridx[r + 1] - ridx[r];
      if (len > 0xFFFFFFFFull) return lz_fail(LZ_EINVAL, "lz_encode: record too long");
      max_rec = std::max<uint32_t>(max_rec, (uint32_t)len);
    }
  }
  Parse ps;
  int rc = pr.segment_log2 ? parse_segmented(x, n, pr, threads, ps)
           : n < (1ull << 32) - 1 ? parse_impl<uint32_t>(x, n, pr, threads, ps)
                                  : parse_impl<uint64_t>(x, n, pr, threads, ps);
  if (rc) return lz_fail(rc, "lz_encode: parse failed");
  rebase_sources(ps, nb, bl, threads);

  // per-block stream bytes, built on demand
  auto build = [&](uint64_t b, std::vector<uint8_t> s[4]) {
    const uint64_t s0 = ps.seq_ptr[b], ns = ps.seq_ptr[b + 1] - s0;
    uint64_t pos = b << bl;
    s[kLit].clear();
    s[kCmd].assign(2 * ns, 0);
    s[kMlen].assign(2 * ns, 0);
    s[kOff].assign(w * ns, 0);
    for (uint64_t j = 0; j < ns; j++) {
      uint32_t L = ps.ll[s0 + j], M = ps.ml[s0 + j];
      uint64_t O = ps.of[s0 + j];
      s[kLit].insert(s[kLit].end(), x + pos, x + pos + L);
      pos += (uint64_t)L + M;
      s[kCmd][j] = (uint8_t)L;
      s[kCmd][ns + j] = (uint8_t)(L >> 8);
      s[kMlen][j] = (uint8_t)M;
      s[kMlen][ns + j] = (uint8_t)(M >> 8);
      for (uint32_t k = 0; k < w; k++) s[kOff][k * ns + j] = (uint8_t)(O >> (8 * k));
    }
  };
  std::vector<std::vector<uint64_t>> cnt(threads, std::vector<uint64_t>(4 * 256, 0));
  parallel_for(nb, threads, [&](uint64_t b, unsigned t) {   // symbol counts of the four streams
    uint64_t* c = cnt[t].data();
    const uint64_t s0 = ps.seq_ptr[b], ns = ps.seq_ptr[b + 1] - s0;
    uint64_t pos = b << bl;
    for (uint64_t j = 0; j < ns; j++) {
      const uint32_t L = ps.ll[s0 + j], M = ps.ml[s0 + j];
      const uint64_t O = ps.of[s0 + j];
      for (uint64_t i = 0; i < L; i++) c[kLit * 256 + x[pos + i]]++;
      pos += (uint64_t)L + M;
      c[kCmd * 256 + (L & 0xFF)]++;
      c[kCmd * 256 + ((L >> 8) & 0xFF)]++;
      c[kMlen * 256 + (M & 0xFF)]++;
      c[kMlen * 256 + ((M >> 8) & 0xFF)]++;
      for (uint32_t k = 0; k < w; k++) c[kOff * 256 + ((O >> (8 * k)) & 0xFF)]++;
    }
  });
  Table tab[4];
  for (int k = 0; k < 4; k++) {
    uint64_t c[256] = {0};
    for (unsigned t = 0; t < threads; t++)
      for (int s = 0; s < 256; s++) c[s] += cnt[t][k * 256 + s];
    tab[k].P = pr.prob_bits[k];
    if (normalize(c, tab[k].P, tab[k].f)) return lz_fail(LZ_EINVAL, "lz_encode: cannot normalise table");
    tab[k].c[0] = 0;
    for (int s = 0; s < 256; s++) tab[k].c[s + 1] = tab[k].c[s] + tab[k].f[s];
  }
  // per-block payloads in parallel
  std::vector<std::vector<uint8_t>> pay(nb);
  std::vector<uint64_t> bh(nb);
  std::vector<uint32_t> nlit(nb);
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    std::vector<uint8_t> s[4];
    build(b, s);
    static const int order[4] = {kCmd, kMlen, kOff, kLit};
    for (int k : order)
      put_stream(pay[b], s[k].data(), (uint32_t)s[k].size(), tab[k], k == kLit ? pr.lit_lanes : pr.seq_lanes,
                 k == kLit ? 16u : 4u);
    const uint64_t sb = b << bl, eb = std::min(sb + B, n);
    bh[b] = fnv1a(x + sb, eb - sb, kFnvBasis);
    nlit[b] = (uint32_t)s[kLit].size();
  });
  // layout
  auto al16 = [](uint64_t v) { return (v + 15) & ~15ull; };
  const uint64_t ndeps = ps.dep_idx.size();
  const uint64_t off_tables = kHeaderSize;
  const uint64_t off_dir = off_tables + kTablesLen;
  const uint64_t off_dep_ptr = al16(off_dir + nb * kDirEntry);
  const uint64_t off_dep_idx = off_dep_ptr + 8 * (nb + 1);
  const uint64_t off_payload = al16(off_dep_idx + 4 * ndeps);
  std::vector<uint64_t> poff(nb + 1, 0);
  for (uint64_t b = 0; b < nb; b++) poff[b + 1] = poff[b] + pay[b].size();
  const uint64_t off_ridx = pr.kind == 1 ? al16(off_payload + poff[nb]) : 0;
  const uint64_t total = pr.kind == 1 ? off_ridx + 8 * ridx.size() : al16(off_payload + poff[nb]);
  uint8_t* A = (uint8_t*)std::calloc(total ? total : 1, 1);
  if (!A) return lz_fail(LZ_EINVAL, "lz_encode: out of host memory");
  for (int k = 0; k < 4; k++) std::memcpy(A + off_tables + 512 * k, tab[k].f, 512);
  uint32_t n_levels = 0;
  for (uint64_t b = 0; b < nb; b++) {
    uint8_t* e = A + off_dir + b * kDirEntry;
    uint32_t ns = (uint32_t)(ps.seq_ptr[b + 1] - ps.seq_ptr[b]), pl = (uint32_t)pay[b].size();
    std::memcpy(e + 0, &poff[b], 8);
    std::memcpy(e + 8, &pl, 4);
    std::memcpy(e + 12, &ns, 4);
    std::memcpy(e + 16, &nlit[b], 4);
    std::memcpy(e + 20, &ps.level[b], 2);
    std::memcpy(e + 24, &bh[b], 8);
    n_levels = std::max<uint32_t>(n_levels, ps.level[b] + 1u);
  }
  std::memcpy(A + off_dep_ptr, ps.dep_ptr.data(), 8 * (nb + 1));
  if (ndeps) std::memcpy(A + off_dep_idx, ps.dep_idx.data(), 4 * ndeps);
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    std::memcpy(A + off_payload + poff[b], pay[b].data(), pay[b].size());
  });
  if (pr.kind == 1) std::memcpy(A + off_ridx, ridx.data(), 8 * ridx.size());
  uint64_t tree = kFnvBasis;
  for (uint64_t b = 0; b < nb; b++) tree = fnv1a((const uint8_t*)&bh[b], 8, tree);
  // header
  uint8_t* h = A;
  std::memcpy(h, "LZAB", 4);
  uint16_t ver = 2, flags = (uint16_t)((pr.kind == 1 ? 1u : 0u) | (pr.level_penalty << 8));
  std::memcpy(h + 4, &ver, 2);
  std::memcpy(h + 6, &flags, 2);
  h[8] = (uint8_t)bl;
  h[9] = (uint8_t)pr.max_level;
  h[10] = (uint8_t)w;
  h[11] = (uint8_t)pr.min_match;
  h[12] = (uint8_t)pr.hash_len;
  h[13] = (uint8_t)pr.kind;
  h[14] = (uint8_t)(pr.lit_lanes - 1);
  h[15] = (uint8_t)pr.seq_lanes;
  for (int k = 0; k < 4; k++) h[16 + k] = (uint8_t)pr.prob_bits[k];
  h[20] = (uint8_t)pr.hash_bits;
  h[21] = (uint8_t)pr.window_log2;
  uint16_t cd = (uint16_t)pr.chain_depth;
  std::memcpy(h + 22, &cd, 2);
  uint64_t n_reads = ridx.empty() ? 0 : ridx.size() - 1;
  uint64_t f64[] = {n, nb, n_reads};
  std::memcpy(h + 24, f64, 24);
  std::memcpy(h + 48, &max_rec, 4);
  std::memcpy(h + 52, &n_levels, 4);
  uint64_t offs[] = {off_tables, off_dir, off_dep_ptr, off_dep_idx, off_payload, off_ridx, total, tree};
  std::memcpy(h + 56, offs, 64);
  uint64_t hf = fnv1a(h, 120, kFnvBasis);
  std::memcpy(h + 120, &hf, 8);
  *archive = A;
  *archive_len = total;
  return LZ_OK;
}

// .fai-style description of the sequences of a FASTA text.  Record starts
// ('>' at the start of a line) are found first; then each sequence's lines
// are checked in parallel chunks: with W the length of its first line, every
// newline but the sequence's last must lie at offset + W + k (W + 1).
extern "C" int lz_fasta_index(const uint8_t* x, uint64_t n, lz_fasta_seq* out, uint64_t cap,
                              uint64_t* count) {
  if (!count || (n && !x) || (cap && !out)) return lz_fail(LZ_EINVAL, "lz_fasta_index: null argument");
  *count = 0;
  if (!n) return LZ_OK;
  if (x[0] != '>') return lz_fail(LZ_EINVAL, "lz_fasta_index: text does not start with '>'");
  std::vector<uint64_t> starts;
  for (uint64_t p = 0; p < n;) {
    const uint8_t* g = (const uint8_t*)std::memchr(x + p, '>', (size_t)(n - p));
    if (!g) break;
    const uint64_t q = (uint64_t)(g - x);
    if (q == 0 || x[q - 1] == '\n') starts.push_back(q);
    p = q + 1;
  }
  starts.push_back(n);
  const unsigned threads = std::max(1u, std::thread::hardware_concurrency());
  for (size_t r = 0; r + 1 < starts.size(); r++) {
    const uint64_t h0 = starts[r], end = starts[r + 1];
    const uint8_t* nl = (const uint8_t*)std::memchr(x + h0, '\n', (size_t)(end - h0));
    const uint64_t he = nl ? (uint64_t)(nl - x) : end;
    lz_fasta_seq sq;
    std::memset(&sq, 0, sizeof(sq));
    uint64_t q = h0 + 1, j = 0;
    while (q < he && x[q] != ' ' && x[q] != '\t' && x[q] != '\r') {
      if (j < sizeof(sq.name) - 1) sq.name[j++] = (char)x[q];
      q++;
    }
    const uint64_t a = std::min(he + 1, end);
    sq.offset = a;
    // first line width, then the other newlines on the grid, in chunks
    const uint8_t* f = (const uint8_t*)std::memchr(x + a, '\n', (size_t)(end - a));
    const uint64_t W = f ? (uint64_t)(f - x) - a : end - a;
    const uint64_t last_nl = (end > a && x[end - 1] == '\n') ? end - 1 : end;   // the sequence's last newline
    const uint64_t chunk = 64ull << 20, nch = (end - a + chunk - 1) / chunk;
    std::vector<uint64_t> nls(nch ? nch : 1, 0);
    std::vector<uint8_t> bad(nch ? nch : 1, 0);
    parallel_for(nch, threads, [&](uint64_t c, unsigned) {
      const uint64_t c0 = a + c * chunk, c1 = std::min(end, c0 + chunk);
      uint64_t cnt = 0;
      for (uint64_t p = c0; p < c1;) {
        const uint8_t* l = (const uint8_t*)std::memchr(x + p, '\n', (size_t)(c1 - p));
        if (!l) break;
        const uint64_t e = (uint64_t)(l - x);
        cnt++;
        if (e != last_nl && (e < a + W || (e - a - W) % (W + 1))) bad[c] = 1;
        p = e + 1;
      }
      nls[c] = cnt;
    });
    uint64_t newlines = 0;
    bool even = W > 0;
    for (uint64_t c = 0; c < nch; c++) { newlines += nls[c]; if (bad[c]) even = false; }
    sq.length = (end - a) - newlines;
    if (even && last_nl == end - 1 && end - 1 > a) {          // last line: 1..W bases
      const uint64_t full = (last_nl - a) / (W + 1), rem = (last_nl - a) - full * (W + 1);
      if (rem > W || (rem == 0 && full == 0)) even = false;
    }
    if (last_nl != end - 1) even = false;                    // text must end its lines with '\n'
    sq.line_bases = even ? (uint32_t)W : 0;
    sq.line_bytes = even ? (uint32_t)(W + 1) : 0;
    if (r < cap) out[r] = sq;
  }
  *count = starts.size() - 1;
  return LZ_OK;
}
