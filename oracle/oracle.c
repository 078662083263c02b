/*
 * Plain CPU oracle: TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written for reading, not speed: byte loops, full-size tables, no blocking,
 * no fusion.  Each section names the paper passage (or the reading of it) that
 * it follows.  Container format v2 is defined by the code below and by the
 * design notes; nothing here is shared with the HIP library.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HDR_SIZE   128
#define DIR_ENTRY  32
#define TABLES_LEN (4 * 256 * 2)
#define MODE_EMPTY 0
#define MODE_CONST 1
#define MODE_RAW   2
#define MODE_RANS  3
#define RANS_L     (1ull << 16)       /* lower bound of the 32-bit state      */
#define FNV_BASIS  0xcbf29ce484222325ull
#define FNV_PRIME  0x00000100000001b3ull
#define GOLDEN     0x9E3779B97F4A7C15ull  /* floor(2^64 / golden ratio)      */

enum { K_LIT = 0, K_CMD = 1, K_MLEN = 2, K_OFF = 3 };

/* ------------------------------------------------------------------ bytes */
static void put16(uint8_t* p, uint64_t v) { for (int k = 0; k < 2; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put32(uint8_t* p, uint64_t v) { for (int k = 0; k < 4; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put64(uint8_t* p, uint64_t v) { for (int k = 0; k < 8; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static uint64_t getn(const uint8_t* p, int n) {
  uint64_t v = 0;
  for (int k = 0; k < n; k++) v |= (uint64_t)p[k] << (8 * k);
  return v;
}
#define get16(p) ((uint32_t)getn((p), 2))
#define get32(p) ((uint32_t)getn((p), 4))
#define get64(p) getn((p), 8)

typedef struct { uint8_t* p; uint64_t n, cap; } buf_t;

static int buf_reserve(buf_t* b, uint64_t extra) {
  if (b->n + extra <= b->cap) return 0;
  uint64_t c = b->cap ? b->cap : 4096;
  while (c < b->n + extra) c *= 2;
  uint8_t* q = (uint8_t*)realloc(b->p, c);
  if (!q) return -1;
  b->p = q;
  b->cap = c;
  return 0;
}
static int buf_put(buf_t* b, const void* d, uint64_t n) {
  if (buf_reserve(b, n)) return -1;
  if (n) memcpy(b->p + b->n, d, n);
  b->n += n;
  return 0;
}
static int buf_zero(buf_t* b, uint64_t n) {
  if (buf_reserve(b, n)) return -1;
  memset(b->p + b->n, 0, n);
  b->n += n;
  return 0;
}
static int buf_pad16(buf_t* b) { return buf_zero(b, (16 - (b->n & 15)) & 15); }

void orc_free(void* p) { free(p); }

/* ------------------------------------------------------------------- FNV
 * FNV-1a-64 with the published offset basis and prime (Experimental Setup:
 * device paths are checked with FNV).  Block tree: FNV-1a-64 over the
 * concatenated little-endian 64-bit block hashes. */
uint64_t orc_fnv_basis(void) { return FNV_BASIS; }
uint64_t orc_fnv1a64(const uint8_t* p, uint64_t n, uint64_t h) {
  for (uint64_t i = 0; i < n; i++) { h ^= p[i]; h *= FNV_PRIME; }
  return h;
}

void orc_params_default(orc_params* p) {
  p->block_log2 = 14;      /* 16 KB blocks (Block Granularity section)      */
  p->max_level = 64;       /* dependency wavefronts up to depth 64          */
  p->min_match = 16;
  p->hash_len = 16;
  p->hash_bits = 20;
  p->chain_depth = 64;
  p->window_log2 = 0;      /* global search: no window                      */
  p->lit_lanes = 256;
  p->seq_lanes = 64;
  p->prob_bits[0] = 12;
  p->prob_bits[1] = p->prob_bits[2] = p->prob_bits[3] = 10;
  p->kind = 0;
  p->level_penalty = 0;
}

/* ------------------------------------------------------- entropy (rANS)
 * The paper only names its entropy stage (an ANS coder); this follows the
 * published rANS of Duda (2013) with the lane interleaving of Giesen (2014):
 * 32-bit state x in [2^16, 2^32), 16-bit renormalisation words, one static
 * normalised frequency table per stream kind per archive. */

/* Normalise counts to sum 2^P: floor(c*M/T) with a floor of 1 for every seen
 * symbol; a positive remainder goes to the most frequent symbol (ties: lowest
 * value); an excess is taken one unit at a time from the largest f > 1 (ties:
 * lowest value). */
int orc_normalize(const uint64_t* counts, uint32_t P, uint16_t* freq) {
  uint64_t T = 0;
  for (int s = 0; s < 256; s++) T += counts[s];
  memset(freq, 0, 256 * sizeof(uint16_t));
  if (T == 0) return ORC_OK;
  if (P < 1 || P > 12) return ORC_EINVAL;
  uint64_t M = 1ull << P;
  int64_t sum = 0;
  for (int s = 0; s < 256; s++) {
    if (!counts[s]) continue;
    uint64_t f = counts[s] * M / T;
    if (f < 1) f = 1;
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
    if (best < 0) return ORC_EINVAL;
    freq[best]--;
    d++;
  }
  return ORC_OK;
}

/* Lanes of a stream of n symbols: the largest power of two <= n/s, at least
 * 1, at most max_lanes, with s = 16 symbols per lane for the literal stream
 * and s = 4 for the (short) CMD, MLEN and OFF streams. */
int orc_rans_lanes(uint32_t n, uint32_t max_lanes, uint32_t per_lane) {
  uint32_t q = n / per_lane, k = 1;
  while (k * 2 <= q) k *= 2;
  return (int)(k < max_lanes ? k : max_lanes);
}

static void cumulative(const uint16_t* freq, uint32_t* cum) {
  cum[0] = 0;
  for (int s = 0; s < 256; s++) cum[s + 1] = cum[s] + freq[s];
}

/* Lane layout: lane k of K holds one run of consecutive symbols.  With
 * R = n / K and e = n mod K, lane k holds len_k = R + (k < e) symbols starting
 * at start_k = k R + min(k, e).  Decoding goes in rounds: in round r every lane
 * with r < len_k decodes its symbol start_k + r; the decoder's slot of (r, k)
 * is r K + k. */
static uint32_t run_len(uint32_t k, uint32_t R, uint32_t e) { return R + (k < e ? 1u : 0u); }
static uint64_t run_start(uint32_t k, uint32_t R, uint32_t e) {
  return (uint64_t)k * R + (k < e ? k : e);
}

/* Encode in the reverse of the decoder's order (rounds from last to first,
 * lanes from K-1 to 0).  Before encoding s a lane whose state is
 * >= f_s * 2^(32-P) emits its low 16 bits.  Body: u32 final state per lane,
 * u32 word count per 64-lane group, then each group's words in the decoder's
 * slot order. */
int orc_rans_encode(const uint8_t* sym, uint32_t n, const uint16_t* freq,
                    uint32_t P, uint32_t K, uint8_t** body, uint64_t* body_len,
                    uint32_t* n_words) {
  if (K < 1 || K > 256 || P < 1 || P > 12) return ORC_EINVAL;
  uint32_t cum[257];
  cumulative(freq, cum);
  if (cum[256] != (1u << P)) return ORC_EINVAL;
  for (uint32_t i = 0; i < n; i++)
    if (!freq[sym[i]]) return ORC_EINVAL;
  uint32_t G = (K + 63) / 64, R = n / K, e = n % K;
  uint64_t slots = (uint64_t)((n + K - 1) / K) * K;
  uint64_t x[256];
  for (uint32_t k = 0; k < K; k++) x[k] = RANS_L;
  int32_t* word = (int32_t*)malloc((slots ? slots : 1) * sizeof(int32_t));
  if (!word) return ORC_EINVAL;
  for (uint64_t o = slots; o-- > 0;) {
    uint32_t r = (uint32_t)(o / K), k = (uint32_t)(o % K);
    word[o] = -1;
    if (r >= run_len(k, R, e)) continue;
    uint32_t s = sym[run_start(k, R, e) + r], f = freq[s];
    uint64_t xmax = (uint64_t)f << (32 - P);
    if (x[k] >= xmax) {
      word[o] = (int32_t)(x[k] & 0xFFFF);
      x[k] >>= 16;
    }
    x[k] = (x[k] / f) * (1ull << P) + (x[k] % f) + cum[s];
  }
  uint32_t gw[4] = {0, 0, 0, 0}, nw = 0;
  for (uint64_t o = 0; o < slots; o++)
    if (word[o] >= 0) { gw[(o % K) / 64]++; nw++; }
  uint64_t len = 4ull * K + 4ull * G + 2ull * nw;
  uint8_t* out = (uint8_t*)malloc(len ? len : 1);
  if (!out) { free(word); return ORC_EINVAL; }
  uint8_t* q = out;
  for (uint32_t k = 0; k < K; k++, q += 4) put32(q, x[k]);
  for (uint32_t g = 0; g < G; g++, q += 4) put32(q, gw[g]);
  for (uint32_t g = 0; g < G; g++)
    for (uint64_t o = 0; o < slots; o++)
      if (word[o] >= 0 && (o % K) / 64 == g) { put16(q, (uint32_t)word[o]); q += 2; }
  free(word);
  *body = out;
  *body_len = len;
  *n_words = nw;
  return ORC_OK;
}

/* Decode round by round: every lane with a symbol this round decodes it
 * (slot = x mod M; s = symbol owning slot; x = f_s (x >> P) + slot - c_s);
 * then the lanes whose state fell below 2^16 read the next word of their
 * group, in ascending lane order.  Afterwards every state is 2^16 and every
 * word has been read, else the stream is corrupt. */
int orc_rans_decode(const uint8_t* body, uint64_t body_len, uint32_t n,
                    uint32_t n_words, const uint16_t* freq, uint32_t P,
                    uint32_t K, uint8_t* out) {
  if (K < 1 || K > 256 || P < 1 || P > 12) return ORC_EINVAL;
  uint32_t G = (K + 63) / 64;
  if (body_len != 4ull * K + 4ull * G + 2ull * n_words) return ORC_ECORRUPT;
  uint32_t cum[257];
  cumulative(freq, cum);
  uint32_t M = 1u << P;
  if (cum[256] != M) return ORC_ECORRUPT;
  uint8_t* slot_sym = (uint8_t*)malloc(M);
  if (!slot_sym) return ORC_EINVAL;
  for (int s = 0; s < 256; s++)
    for (uint32_t t = cum[s]; t < cum[s + 1]; t++) slot_sym[t] = (uint8_t)s;
  uint64_t x[256];
  for (uint32_t k = 0; k < K; k++) {
    x[k] = get32(body + 4 * k);
    if (x[k] < RANS_L) { free(slot_sym); return ORC_ECORRUPT; }
  }
  uint32_t gw[4], gstart[4], gpos[4], tot = 0;
  for (uint32_t g = 0; g < G; g++) {
    gw[g] = get32(body + 4 * K + 4 * g);
    gstart[g] = tot;
    gpos[g] = 0;
    tot += gw[g];
  }
  if (tot != n_words) { free(slot_sym); return ORC_ECORRUPT; }
  const uint8_t* W = body + 4 * K + 4 * G;
  uint32_t rounds = (n + K - 1) / K, R = n / K, e = n % K;
  int rc = ORC_OK;
  for (uint32_t r = 0; r < rounds && rc == ORC_OK; r++) {
    for (uint32_t k = 0; k < K; k++) {
      if (r >= run_len(k, R, e)) continue;
      uint32_t slot = (uint32_t)(x[k] & (M - 1));
      uint32_t s = slot_sym[slot];
      x[k] = (uint64_t)freq[s] * (x[k] >> P) + slot - cum[s];
      out[run_start(k, R, e) + r] = (uint8_t)s;
    }
    for (uint32_t k = 0; k < K; k++) {
      if (r >= run_len(k, R, e)) continue;
      if (x[k] < RANS_L) {
        uint32_t g = k / 64;
        if (gpos[g] >= gw[g]) { rc = ORC_ECORRUPT; break; }
        x[k] = (x[k] << 16) | get16(W + 2ull * (gstart[g] + gpos[g]));
        gpos[g]++;
      }
    }
  }
  for (uint32_t k = 0; k < K && rc == ORC_OK; k++)
    if (x[k] != RANS_L) rc = ORC_ECORRUPT;
  for (uint32_t g = 0; g < G && rc == ORC_OK; g++)
    if (gpos[g] != gw[g]) rc = ORC_ECORRUPT;
  free(slot_sym);
  return rc;
}

/* --------------------------------------------------------- match search
 * Global match search with absolute source positions (Background section),
 * greedy, with the dependency-level cap.  hash(p) is Fibonacci hashing of the
 * first h bytes at p; every position p with p + h <= N enters a chain in
 * increasing order (head = most recent, prev = link, anchor = first position
 * ever seen for that hash).  At p the candidates are the chain (most recent
 * first, at most C, none older than 2^R) and then the anchor.  A candidate's
 * match length is the common prefix of x[q:] and x[p:], capped at the block
 * end; its level is 0 for a source inside the block, else 1 + the highest
 * level among the earlier blocks its source touches.  Candidates shorter than
 * m or with level > D-1 are dropped; the longest wins, then the lowest level,
 * then the first seen. */
static uint64_t hash_at(const uint8_t* x, uint64_t p, uint32_t h, uint32_t H) {
  uint64_t v0 = 0, v1 = 0;
  uint32_t n0 = h < 8 ? h : 8;
  for (uint32_t k = 0; k < n0; k++) v0 |= (uint64_t)x[p + k] << (8 * k);
  for (uint32_t k = 8; k < h; k++) v1 |= (uint64_t)x[p + k] << (8 * (k - 8));
  uint64_t t = v0 * GOLDEN;
  t = (t << 29) | (t >> 35);
  return ((t ^ v1) * GOLDEN) >> (64 - H);
}

typedef struct {
  uint64_t n, cap;
  uint32_t *blk, *ll, *ml;
  uint64_t* of;
} seqs_t;

static int seq_push(seqs_t* s, uint32_t blk, uint32_t ll, uint32_t ml, uint64_t of) {
  if (s->n == s->cap) {
    uint64_t c = s->cap ? 2 * s->cap : 1024;
    uint32_t* a = (uint32_t*)realloc(s->blk, c * 4);
    if (!a) return -1;
    s->blk = a;
    a = (uint32_t*)realloc(s->ll, c * 4);
    if (!a) return -1;
    s->ll = a;
    a = (uint32_t*)realloc(s->ml, c * 4);
    if (!a) return -1;
    s->ml = a;
    uint64_t* o = (uint64_t*)realloc(s->of, c * 8);
    if (!o) return -1;
    s->of = o;
    s->cap = c;
  }
  s->blk[s->n] = blk;
  s->ll[s->n] = ll;
  s->ml[s->n] = ml;
  s->of[s->n] = of;
  s->n++;
  return 0;
}

typedef struct {
  seqs_t seq;
  uint16_t* level;      /* per block */
  uint64_t* dep_ptr;    /* n_blocks + 1 */
  uint32_t* dep_idx;
  uint64_t n_deps;
} parse_t;

static void parse_free(parse_t* r) {
  free(r->seq.blk); free(r->seq.ll); free(r->seq.ml); free(r->seq.of);
  free(r->level); free(r->dep_ptr); free(r->dep_idx);
  memset(r, 0, sizeof(*r));
}

static int check_params(const orc_params* p) {
  if (p->block_log2 < 6 || p->block_log2 > 15) return ORC_EINVAL;
  if (p->max_level < 1 || p->max_level > 64) return ORC_EINVAL;
  if (p->hash_len < 4 || p->hash_len > 16) return ORC_EINVAL;
  if (p->min_match < p->hash_len || p->min_match > 255) return ORC_EINVAL;
  if (p->hash_bits < 8 || p->hash_bits > 30) return ORC_EINVAL;
  if (p->window_log2 > 40) return ORC_EINVAL;
  if (p->chain_depth > 65535) return ORC_EINVAL;
  if (p->lit_lanes < 1 || p->lit_lanes > 256) return ORC_EINVAL;
  if (p->seq_lanes < 1 || p->seq_lanes > 64) return ORC_EINVAL;
  for (int k = 0; k < 4; k++)
    if (p->prob_bits[k] < 8 || p->prob_bits[k] > 12) return ORC_EINVAL;
  if (p->kind > 2) return ORC_EINVAL;
  if (p->level_penalty > 255) return ORC_EINVAL;
  return ORC_OK;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

static int do_parse(const uint8_t* x, uint64_t n, const orc_params* pr, parse_t* out) {
  memset(out, 0, sizeof(*out));
  const uint64_t B = 1ull << pr->block_log2;
  const uint64_t nb = (n + B - 1) / B;
  const uint32_t h = pr->hash_len, m = pr->min_match, H = pr->hash_bits;
  const uint32_t C = pr->chain_depth, R = pr->window_log2, D = pr->max_level;
  const uint32_t beta = pr->level_penalty;
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) << H);
  int64_t* anchor = (int64_t*)malloc(sizeof(int64_t) << H);
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  out->level = (uint16_t*)calloc(nb ? nb : 1, sizeof(uint16_t));
  out->dep_ptr = (uint64_t*)calloc(nb + 1, sizeof(uint64_t));
  uint8_t* dep_mark = (uint8_t*)calloc(nb ? nb : 1, 1);
  uint32_t* blist = (uint32_t*)malloc((nb ? nb : 1) * sizeof(uint32_t));
  uint64_t nlist = 0;
  uint64_t dep_cap = 1024;
  out->dep_idx = (uint32_t*)malloc(dep_cap * 4);
  if (!head || !anchor || !prev || !out->level || !out->dep_ptr || !dep_mark || !blist || !out->dep_idx) {
    free(head); free(anchor); free(prev); free(dep_mark); free(blist);
    parse_free(out);
    return ORC_EINVAL;
  }
  for (uint64_t i = 0; i < (1ull << H); i++) head[i] = anchor[i] = -1;
  uint64_t next_ins = 0;
  int rc = ORC_OK;
  for (uint64_t b = 0; b < nb && rc == ORC_OK; b++) {
    const uint64_t sb = b * B, eb = (sb + B < n) ? sb + B : n;
    uint64_t p = sb, lit = sb;
    uint32_t blevel = 0;
    while (p < eb) {
      for (; next_ins < p; next_ins++) {
        if (next_ins + h > n) continue;
        uint64_t hv = hash_at(x, next_ins, h, H);
        prev[next_ins] = head[hv];
        head[hv] = (int64_t)next_ins;
        if (anchor[hv] < 0) anchor[hv] = (int64_t)next_ins;
      }
      uint64_t best_L = 0, best_q = 0;
      uint32_t best_lv = 0;
      int64_t best_sc = 0;
      if (p + m <= eb) {
        uint64_t hv = hash_at(x, p, h, H);
        int64_t a = anchor[hv];
        int anchor_seen = 0;
        uint64_t cnt = 0;
        int64_t q = head[hv];
        for (int phase = 0; phase < 2; phase++) {
          while (1) {
            int64_t c;
            if (phase == 0) {
              if (q < 0) break;
              if (C && cnt >= C) break;
              if (R && (uint64_t)(p - (uint64_t)q) > (1ull << R)) break;
              c = q;
              if (q == a) anchor_seen = 1;
              q = prev[q];
              cnt++;
            } else {
              if (a < 0 || anchor_seen) break;
              c = a;
              anchor_seen = 1;
            }
            uint64_t cq = (uint64_t)c;
            uint64_t cap = eb - p, L = 0;
            while (L < cap && x[cq + L] == x[p + L]) L++;
            if (L < m) continue;
            uint32_t lv = 0;
            if (cq < sb) {
              uint64_t hi = cq + L < sb ? cq + L : sb;
              uint32_t mx = 0;
              for (uint64_t blk = cq >> pr->block_log2; blk <= (hi - 1) >> pr->block_log2; blk++)
                if (out->level[blk] > mx) mx = out->level[blk];
              lv = 1 + mx;
            }
            if (lv > D - 1) continue;
            /* score = L - beta * lv: every level a source adds costs beta
             * bytes of match length; a candidate must score at least m
             * (beta = 0: longest first, then lowest level) */
            int64_t sc = (int64_t)L - (int64_t)beta * lv;
            if (sc < (int64_t)m) continue;
            if (best_L == 0 || sc > best_sc || (sc == best_sc && lv < best_lv)) {
              best_sc = sc;
              best_L = L;
              best_q = cq;
              best_lv = lv;
            }
          }
        }
      }
      if (best_L) {
        if (seq_push(&out->seq, (uint32_t)b, (uint32_t)(p - lit), (uint32_t)best_L, best_q)) { rc = ORC_EINVAL; break; }
        if (best_q < sb) {
          uint64_t hi = best_q + best_L < sb ? best_q + best_L : sb;
          for (uint64_t blk = best_q >> pr->block_log2; blk <= (hi - 1) >> pr->block_log2; blk++)
            if (!dep_mark[blk]) { dep_mark[blk] = 1; blist[nlist++] = (uint32_t)blk; }
        }
        if (best_lv > blevel) blevel = best_lv;
        p += best_L;
        lit = p;
      } else {
        p++;
      }
    }
    if (rc) break;
    if (lit < eb)
      if (seq_push(&out->seq, (uint32_t)b, (uint32_t)(eb - lit), 0, 0)) { rc = ORC_EINVAL; break; }
    out->level[b] = (uint16_t)blevel;
    /* deps(b): the marked earlier blocks in ascending order; clear the marks */
    qsort(blist, nlist, sizeof(uint32_t), cmp_u32);
    for (uint64_t k = 0; k < nlist; k++) {
      dep_mark[blist[k]] = 0;
      if (out->n_deps == dep_cap) {
        dep_cap *= 2;
        uint32_t* t = (uint32_t*)realloc(out->dep_idx, dep_cap * 4);
        if (!t) { rc = ORC_EINVAL; break; }
        out->dep_idx = t;
      }
      out->dep_idx[out->n_deps++] = blist[k];
    }
    nlist = 0;
    out->dep_ptr[b + 1] = out->n_deps;
  }
  free(head); free(anchor); free(prev); free(dep_mark); free(blist);
  if (rc) parse_free(out);
  return rc;
}

int orc_parse(const uint8_t* src, uint64_t n, const orc_params* p, uint64_t* n_seq,
              uint32_t** blk, uint32_t** ll, uint32_t** ml, uint64_t** of,
              uint16_t** level) {
  int rc = check_params(p);
  if (rc) return rc;
  parse_t r;
  rc = do_parse(src, n, p, &r);
  if (rc) return rc;
  *n_seq = r.seq.n;
  *blk = r.seq.blk; *ll = r.seq.ll; *ml = r.seq.ml; *of = r.seq.of;
  *level = r.level;
  free(r.dep_ptr);
  free(r.dep_idx);
  return ORC_OK;
}

/* ---------------------------------------------------------- rebasing
 * An encoder choice the format leaves free (any source position holding the
 * same bytes decodes alike): a match that does not overlap itself and whose
 * source window [o, o + M) lies wholly inside the destination of an earlier
 * match of the same block -- one that does not overlap itself either, so its
 * destination equals its source byte for byte -- takes its bytes from that
 * match's source instead: o becomes o_c + (o - p_c).  This is repeated until
 * no such match holds the window (each step moves to a match of smaller
 * index, so it ends).  Matches are handled in sequence order, so an earlier
 * match's source is already final.  The window moves into a region the block
 * already depends on, so dependencies and levels do not change; in-block
 * copy chains get shorter.  Applied to the sequences of blocks [0, nb). */
void orc_rebase(uint64_t n_seq, const uint32_t* blk, const uint32_t* ll, const uint32_t* ml,
                uint64_t* of, uint32_t block_log2) {
  uint64_t i = 0;
  uint64_t* pd = (uint64_t*)malloc((n_seq ? n_seq : 1) * 8);   /* destinations of the block's matches */
  uint64_t* ix = (uint64_t*)malloc((n_seq ? n_seq : 1) * 8);   /* their sequence indexes */
  while (i < n_seq) {
    uint64_t j = i;
    while (j < n_seq && blk[j] == blk[i]) j++;
    uint64_t pos = (uint64_t)blk[i] << block_log2, nm = 0;
    for (uint64_t q = i; q < j; q++) {
      pos += ll[q];
      if (ml[q]) { pd[nm] = pos; ix[nm] = q; nm++; }
      pos += ml[q];
    }
    for (uint64_t m = 0; m < nm; m++) {
      const uint64_t q = ix[m], p = pd[m], M = ml[q];
      for (;;) {
        const uint64_t o = of[q];
        if (p - o < M) break;                       /* overlaps itself */
        /* the last earlier match whose destination starts at or before o */
        uint64_t lo = 0, hi = m;                     /* answer in [0, m): first with pd > o, minus one */
        while (lo < hi) {
          const uint64_t mid = (lo + hi) / 2;
          if (pd[mid] <= o) lo = mid + 1; else hi = mid;
        }
        if (lo == 0) break;
        const uint64_t c = lo - 1, qc = ix[c], pc = pd[c], Mc = ml[qc], oc = of[qc];
        if (o + M > pc + Mc) break;                 /* window not inside its destination */
        if (pc - oc < Mc) break;                    /* it overlaps itself */
        of[q] = oc + (o - pc);
      }
    }
    i = j;
  }
  free(pd);
  free(ix);
}

/* -------------------------------------------------------------- streams
 * Four streams per block (Background section): CMD = literal-run lengths,
 * MLEN = match lengths, OFF = absolute source offsets, LIT = literal bytes.
 * CMD and MLEN hold u16 values and OFF holds w-byte values, stored byte-plane
 * major (all low bytes, then the next byte of every value, ...), so every
 * stream is a byte string coded with a byte alphabet. */
static int offset_width(uint64_t n) {
  uint64_t v = n ? n - 1 : 0;
  int bits = 0;
  while (v) { bits++; v >>= 1; }
  int w = (bits + 7) / 8;
  return w < 1 ? 1 : w;
}

/* Stream record: 16-byte header {u8 mode, u8 const symbol, u16 lanes,
 * u32 n_sym, u32 n_words, u32 body_len}, body, zero padding to 16 bytes.
 * EMPTY for n = 0, CONST for a single distinct symbol, else rANS unless its
 * body would be >= n bytes, in which case the bytes are stored RAW. */
static int write_stream(buf_t* b, const uint8_t* sym, uint32_t n,
                        const uint16_t* freq, uint32_t P, uint32_t max_lanes,
                        uint32_t per_lane) {
  uint8_t hdr[16];
  memset(hdr, 0, 16);
  put32(hdr + 4, n);
  if (n == 0) {
    hdr[0] = MODE_EMPTY;
    return buf_put(b, hdr, 16);
  }
  int same = 1;
  for (uint32_t i = 1; i < n; i++) if (sym[i] != sym[0]) { same = 0; break; }
  if (same) {
    hdr[0] = MODE_CONST;
    hdr[1] = sym[0];
    return buf_put(b, hdr, 16);
  }
  uint32_t K = (uint32_t)orc_rans_lanes(n, max_lanes, per_lane);
  uint8_t* body = NULL;
  uint64_t blen = 0;
  uint32_t nw = 0;
  int rc = orc_rans_encode(sym, n, freq, P, K, &body, &blen, &nw);
  if (rc) return rc;
  if (blen >= n) {
    hdr[0] = MODE_RAW;
    put32(hdr + 12, n);
    rc = buf_put(b, hdr, 16) || buf_put(b, sym, n) || buf_pad16(b);
  } else {
    hdr[0] = MODE_RANS;
    put16(hdr + 2, K);
    put32(hdr + 8, nw);
    put32(hdr + 12, blen);
    rc = buf_put(b, hdr, 16) || buf_put(b, body, blen) || buf_pad16(b);
  }
  free(body);
  return rc ? ORC_EINVAL : ORC_OK;
}

/* Read index (Read-Level Index section: 8 bytes per read): for FASTQ, the
 * absolute start of line 4r for every read r, then N.  Records are found by
 * counting lines, never by looking for '@' (a quality line may start with
 * '@').  A trailing partial record is rejected. */
static int build_read_index(const uint8_t* x, uint64_t n, uint64_t** idx,
                            uint64_t* n_reads, uint32_t* max_rec) {
  uint64_t lines = 0;
  for (uint64_t i = 0; i < n; i++) lines += (x[i] == '\n');
  if (n && x[n - 1] != '\n') return ORC_EINVAL;
  if (lines % 4) return ORC_EINVAL;
  uint64_t nr = lines / 4;
  uint64_t* r = (uint64_t*)malloc((nr + 1) * 8);
  if (!r) return ORC_EINVAL;
  uint64_t line = 0, mx = 0;
  r[0] = 0;
  for (uint64_t i = 0; i < n; i++) {
    if (x[i] != '\n') continue;
    line++;
    if (line % 4 == 0) r[line / 4] = i + 1;
  }
  for (uint64_t k = 0; k < nr; k++)
    if (r[k + 1] - r[k] > mx) mx = r[k + 1] - r[k];
  if (mx > 0xFFFFFFFFull) { free(r); return ORC_EINVAL; }
  *idx = r;
  *n_reads = nr;
  *max_rec = (uint32_t)mx;
  return ORC_OK;
}

int orc_encode(const uint8_t* x, uint64_t n, const orc_params* pr,
               uint8_t** archive, uint64_t* archive_len) {
  int rc = check_params(pr);
  if (rc) return rc;
  const uint64_t B = 1ull << pr->block_log2;
  const uint64_t nb = (n + B - 1) / B;
  const int w = offset_width(n);
  uint64_t* ridx = NULL;
  uint64_t n_reads = 0;
  uint32_t max_rec = 0;
  if (pr->kind == 1) {
    rc = build_read_index(x, n, &ridx, &n_reads, &max_rec);
    if (rc) return rc;
  }
  parse_t ps;
  rc = do_parse(x, n, pr, &ps);
  if (rc) { free(ridx); return rc; }
  orc_rebase(ps.seq.n, ps.seq.blk, ps.seq.ll, ps.seq.ml, ps.seq.of, pr->block_log2);

  /* per-block sequence ranges */
  uint64_t* sptr = (uint64_t*)calloc(nb + 1, 8);
  for (uint64_t i = 0; i < ps.seq.n; i++) sptr[ps.seq.blk[i] + 1]++;
  for (uint64_t b = 0; b < nb; b++) sptr[b + 1] += sptr[b];

  /* streams of one block into caller buffers; returns lengths */
  uint64_t counts[4][256];
  memset(counts, 0, sizeof(counts));
  uint8_t* sbuf[4];
  sbuf[K_LIT] = (uint8_t*)malloc(B);
  uint64_t max_seq_blk = 0;
  for (uint64_t b = 0; b < nb; b++)
    if (sptr[b + 1] - sptr[b] > max_seq_blk) max_seq_blk = sptr[b + 1] - sptr[b];
  sbuf[K_CMD] = (uint8_t*)malloc(2 * max_seq_blk + 1);
  sbuf[K_MLEN] = (uint8_t*)malloc(2 * max_seq_blk + 1);
  sbuf[K_OFF] = (uint8_t*)malloc((uint64_t)w * max_seq_blk + 1);
  uint32_t slen[4];

#define BUILD_BLOCK(b)                                                          \
  do {                                                                          \
    uint64_t s0 = sptr[b], ns = sptr[(b) + 1] - sptr[b];                        \
    uint64_t pos = (uint64_t)(b) * B, nl = 0;                                   \
    for (uint64_t j = 0; j < ns; j++) {                                         \
      uint32_t L = ps.seq.ll[s0 + j], Mm = ps.seq.ml[s0 + j];                   \
      uint64_t O = ps.seq.of[s0 + j];                                           \
      memcpy(sbuf[K_LIT] + nl, x + pos, L);                                     \
      nl += L;                                                                  \
      pos += (uint64_t)L + Mm;                                                  \
      sbuf[K_CMD][j] = (uint8_t)L;                                              \
      sbuf[K_CMD][ns + j] = (uint8_t)(L >> 8);                                  \
      sbuf[K_MLEN][j] = (uint8_t)Mm;                                            \
      sbuf[K_MLEN][ns + j] = (uint8_t)(Mm >> 8);                                \
      for (int k = 0; k < w; k++) sbuf[K_OFF][k * ns + j] = (uint8_t)(O >> (8 * k)); \
    }                                                                           \
    slen[K_LIT] = (uint32_t)nl;                                                 \
    slen[K_CMD] = slen[K_MLEN] = (uint32_t)(2 * ns);                            \
    slen[K_OFF] = (uint32_t)(w * ns);                                           \
  } while (0)

  for (uint64_t b = 0; b < nb; b++) {
    BUILD_BLOCK(b);
    for (int k = 0; k < 4; k++)
      for (uint32_t i = 0; i < slen[k]; i++) counts[k][sbuf[k][i]]++;
  }
  uint16_t freq[4][256];
  for (int k = 0; k < 4 && !rc; k++) rc = orc_normalize(counts[k], pr->prob_bits[k], freq[k]);

  buf_t pay = {0, 0, 0};
  uint8_t* dir = (uint8_t*)calloc(nb ? nb : 1, DIR_ENTRY);
  uint64_t* bh = (uint64_t*)malloc((nb ? nb : 1) * 8);
  static const int order[4] = {K_CMD, K_MLEN, K_OFF, K_LIT};
  for (uint64_t b = 0; b < nb && !rc; b++) {
    BUILD_BLOCK(b);
    uint64_t start = pay.n;
    for (int t = 0; t < 4 && !rc; t++) {
      int k = order[t];
      rc = write_stream(&pay, sbuf[k], slen[k], freq[k], pr->prob_bits[k],
                        k == K_LIT ? pr->lit_lanes : pr->seq_lanes, k == K_LIT ? 16 : 4);
    }
    uint64_t sb = b * B, eb = sb + B < n ? sb + B : n;
    bh[b] = orc_fnv1a64(x + sb, eb - sb, FNV_BASIS);
    uint8_t* e = dir + b * DIR_ENTRY;
    put64(e + 0, start);
    put32(e + 8, pay.n - start);
    put32(e + 12, sptr[b + 1] - sptr[b]);
    put32(e + 16, slen[K_LIT]);
    put16(e + 20, ps.level[b]);
    put16(e + 22, 0);
    put64(e + 24, bh[b]);
  }
#undef BUILD_BLOCK
  uint32_t n_levels = 0;
  for (uint64_t b = 0; b < nb; b++)
    if ((uint32_t)ps.level[b] + 1 > n_levels) n_levels = ps.level[b] + 1u;
  uint8_t tmp8[8];
  uint64_t tree = FNV_BASIS;
  for (uint64_t b = 0; b < nb; b++) { put64(tmp8, bh[b]); tree = orc_fnv1a64(tmp8, 8, tree); }

  buf_t A = {0, 0, 0};
  if (!rc) {
    rc = buf_zero(&A, HDR_SIZE) ? ORC_EINVAL : ORC_OK;
    uint64_t off_tables = A.n;
    for (int k = 0; k < 4 && !rc; k++)
      for (int s = 0; s < 256; s++) { put16(tmp8, freq[k][s]); rc = buf_put(&A, tmp8, 2) ? ORC_EINVAL : 0; }
    uint64_t off_dir = A.n;
    if (!rc) rc = buf_put(&A, dir, nb * DIR_ENTRY) || buf_pad16(&A) ? ORC_EINVAL : 0;
    uint64_t off_dep_ptr = A.n;
    for (uint64_t b = 0; b <= nb && !rc; b++) { put64(tmp8, ps.dep_ptr[b]); rc = buf_put(&A, tmp8, 8) ? ORC_EINVAL : 0; }
    uint64_t off_dep_idx = A.n;
    for (uint64_t i = 0; i < ps.n_deps && !rc; i++) { put32(tmp8, ps.dep_idx[i]); rc = buf_put(&A, tmp8, 4) ? ORC_EINVAL : 0; }
    if (!rc) rc = buf_pad16(&A) ? ORC_EINVAL : 0;
    uint64_t off_payload = A.n;
    if (!rc) rc = buf_put(&A, pay.p, pay.n) || buf_pad16(&A) ? ORC_EINVAL : 0;
    uint64_t off_ridx = 0;
    if (!rc && pr->kind == 1) {
      off_ridx = A.n;
      for (uint64_t r = 0; r <= n_reads && !rc; r++) { put64(tmp8, ridx[r]); rc = buf_put(&A, tmp8, 8) ? ORC_EINVAL : 0; }
    }
    if (!rc) {
      uint8_t* h = A.p;
      memcpy(h, "LZAB", 4);
      put16(h + 4, 2);
      put16(h + 6, (pr->kind == 1 ? 1u : 0u) | (pr->level_penalty << 8));
      h[8] = (uint8_t)pr->block_log2;
      h[9] = (uint8_t)pr->max_level;
      h[10] = (uint8_t)w;
      h[11] = (uint8_t)pr->min_match;
      h[12] = (uint8_t)pr->hash_len;
      h[13] = (uint8_t)pr->kind;
      h[14] = (uint8_t)(pr->lit_lanes - 1);
      h[15] = (uint8_t)pr->seq_lanes;
      for (int k = 0; k < 4; k++) h[16 + k] = (uint8_t)pr->prob_bits[k];
      h[20] = (uint8_t)pr->hash_bits;
      h[21] = (uint8_t)pr->window_log2;
      put16(h + 22, pr->chain_depth);
      put64(h + 24, n);
      put64(h + 32, nb);
      put64(h + 40, n_reads);
      put32(h + 48, max_rec);
      put32(h + 52, n_levels);
      put64(h + 56, off_tables);
      put64(h + 64, off_dir);
      put64(h + 72, off_dep_ptr);
      put64(h + 80, off_dep_idx);
      put64(h + 88, off_payload);
      put64(h + 96, off_ridx);
      put64(h + 104, A.n);
      put64(h + 112, tree);
      put64(h + 120, orc_fnv1a64(h, 120, FNV_BASIS));
    }
  }
  free(pay.p); free(dir); free(bh); free(sptr); free(ridx);
  for (int k = 0; k < 4; k++) free(sbuf[k]);
  parse_free(&ps);
  if (rc) { free(A.p); return rc; }
  *archive = A.p;
  *archive_len = A.n;
  return ORC_OK;
}

/* ------------------------------------------------------------ container */
typedef struct {
  const uint8_t* a;
  uint64_t len, n, nb, n_reads, tables, dir, dep_ptr, dep_idx, payload, ridx,
      total, tree;
  uint32_t bl, D, w, m, kind, lit_lanes, seq_lanes, n_levels, max_rec;
  uint32_t P[4];
  uint16_t freq[4][256];
} view_t;

static int in_bounds(uint64_t off, uint64_t sz, uint64_t len) {
  return off <= len && sz <= len - off;
}

/* Header and section-bound checks (magic, version, header checksum, field
 * ranges, n_blocks = ceil(N/B), canonical offset width, section layout). */
static int open_view(const uint8_t* a, uint64_t len, view_t* v) {
  memset(v, 0, sizeof(*v));
  if (!a || len < HDR_SIZE) return ORC_EFORMAT;
  if (memcmp(a, "LZAB", 4) || get16(a + 4) != 2) return ORC_EFORMAT;
  if (get64(a + 120) != orc_fnv1a64(a, 120, FNV_BASIS)) return ORC_EFORMAT;
  v->a = a;
  v->len = len;
  v->bl = a[8]; v->D = a[9]; v->w = a[10]; v->m = a[11]; v->kind = a[13];
  v->lit_lanes = a[14] + 1u; v->seq_lanes = a[15];
  for (int k = 0; k < 4; k++) v->P[k] = a[16 + k];
  v->n = get64(a + 24); v->nb = get64(a + 32); v->n_reads = get64(a + 40);
  v->max_rec = get32(a + 48); v->n_levels = get32(a + 52);
  v->tables = get64(a + 56); v->dir = get64(a + 64); v->dep_ptr = get64(a + 72);
  v->dep_idx = get64(a + 80); v->payload = get64(a + 88); v->ridx = get64(a + 96);
  v->total = get64(a + 104); v->tree = get64(a + 112);
  if (v->total != len) return ORC_EFORMAT;
  if (v->bl < 6 || v->bl > 15 || v->D < 1 || v->D > 64) return ORC_EFORMAT;
  if (v->seq_lanes < 1 || v->seq_lanes > 64 || v->kind > 2 || v->m < 1) return ORC_EFORMAT;
  for (int k = 0; k < 4; k++) if (v->P[k] < 8 || v->P[k] > 12) return ORC_EFORMAT;
  if ((int)v->w != offset_width(v->n)) return ORC_EFORMAT;
  if (v->nb != (v->n + (1ull << v->bl) - 1) >> v->bl) return ORC_EFORMAT;
  if (v->nb > 0xFFFFFFFFull) return ORC_EFORMAT;
  if (v->tables != HDR_SIZE || !in_bounds(v->tables, TABLES_LEN, len)) return ORC_EFORMAT;
  if (v->dir < v->tables + TABLES_LEN || !in_bounds(v->dir, v->nb * DIR_ENTRY, len)) return ORC_EFORMAT;
  if (v->dep_ptr < v->dir + v->nb * DIR_ENTRY || !in_bounds(v->dep_ptr, (v->nb + 1) * 8, len)) return ORC_EFORMAT;
  if (v->dep_idx < v->dep_ptr + (v->nb + 1) * 8 || v->dep_idx > len) return ORC_EFORMAT;
  uint64_t ndeps = get64(a + v->dep_ptr + 8 * v->nb);
  if (!in_bounds(v->dep_idx, ndeps * 4, len)) return ORC_EFORMAT;
  if (v->payload < v->dep_idx + ndeps * 4 || v->payload > len) return ORC_EFORMAT;
  uint32_t flags = get16(a + 6);
  if ((flags & 1) != (v->kind == 1) || (flags & 0xFE)) return ORC_EFORMAT;
  if (flags & 1) {
    if (v->ridx < v->payload || !in_bounds(v->ridx, (v->n_reads + 1) * 8, len)) return ORC_EFORMAT;
  } else if (v->ridx != 0 || v->n_reads != 0) {
    return ORC_EFORMAT;
  }
  for (int k = 0; k < 4; k++) {
    uint32_t sum = 0;
    for (int s = 0; s < 256; s++) {
      v->freq[k][s] = (uint16_t)get16(a + v->tables + 512 * k + 2 * s);
      sum += v->freq[k][s];
    }
    if (sum != 0 && sum != (1u << v->P[k])) return ORC_EFORMAT;
  }
  return ORC_OK;
}

/* Full validation: directory (payload ranges, level < D), dependency CSR
 * (ascending, every dependency earlier than its block), level of every block
 * = 0 without dependencies else 1 + max level of its dependencies, n_levels,
 * read index (starts at 0, strictly increasing, ends at N). */
int orc_validate(const uint8_t* a, uint64_t len) {
  view_t v;
  int rc = open_view(a, len, &v);
  if (rc) return rc;
  const uint64_t paylen = (v.kind == 1 ? v.ridx : len) - v.payload;
  uint32_t maxlv = 0;
  uint64_t prev_end = 0;
  for (uint64_t b = 0; b < v.nb; b++) {
    const uint8_t* e = a + v.dir + b * DIR_ENTRY;
    uint64_t po = get64(e), pl = get32(e + 8);
    uint32_t lv = get16(e + 20);
    if (po < prev_end || !in_bounds(po, pl, paylen)) return ORC_EFORMAT;
    prev_end = po + pl;
    if (lv >= v.D) return ORC_EFORMAT;
    if (get32(e + 12) < 1) return ORC_EFORMAT;
    uint64_t d0 = get64(a + v.dep_ptr + 8 * b), d1 = get64(a + v.dep_ptr + 8 * (b + 1));
    if ((b == 0 && d0 != 0) || d1 < d0) return ORC_EFORMAT;
    uint32_t want = 0;
    int64_t last = -1;
    for (uint64_t k = d0; k < d1; k++) {
      uint64_t d = get32(a + v.dep_idx + 4 * k);
      if ((int64_t)d <= last || d >= b) return ORC_EFORMAT;
      last = (int64_t)d;
      uint32_t dl = get16(a + v.dir + d * DIR_ENTRY + 20);
      if (dl + 1 > want) want = dl + 1;
    }
    if (lv != want) return ORC_EFORMAT;
    if (lv > maxlv) maxlv = lv;
  }
  if (v.n_levels != (v.nb ? maxlv + 1 : 0)) return ORC_EFORMAT;
  if (v.kind == 1) {
    uint64_t prev = get64(a + v.ridx);
    if (prev != 0) return ORC_EFORMAT;
    uint64_t mx = 0;
    for (uint64_t r = 1; r <= v.n_reads; r++) {
      uint64_t c = get64(a + v.ridx + 8 * r);
      if (c <= prev) return ORC_EFORMAT;
      if (c - prev > mx) mx = c - prev;
      prev = c;
    }
    if (prev != v.n || mx != v.max_rec) return ORC_EFORMAT;
  }
  return ORC_OK;
}

int orc_info_get(const uint8_t* a, uint64_t len, orc_info* o) {
  view_t v;
  int rc = open_view(a, len, &v);
  if (rc) return rc;
  o->n = v.n; o->n_blocks = v.nb; o->n_reads = v.n_reads; o->total_len = v.total;
  o->source_fnv = v.tree; o->block_log2 = v.bl; o->max_level = v.D;
  o->n_levels = v.n_levels; o->offset_width = v.w; o->max_record_len = v.max_rec;
  o->kind = v.kind;
  return ORC_OK;
}

/* Decode one stream record at payload offset *off (advanced past it). */
static int read_stream(const view_t* v, int kind, const uint8_t* blk,
                       uint64_t blen, uint64_t* off, uint32_t want_n, uint8_t* out) {
  if (!in_bounds(*off, 16, blen)) return ORC_ECORRUPT;
  const uint8_t* h = blk + *off;
  uint32_t mode = h[0], K = get16(h + 2), n = get32(h + 4), nw = get32(h + 8), bl = get32(h + 12);
  if (n != want_n) return ORC_ECORRUPT;
  uint64_t body = *off + 16;
  int rc = ORC_OK;
  switch (mode) {
    case MODE_EMPTY:
      if (n != 0 || bl != 0) return ORC_ECORRUPT;
      break;
    case MODE_CONST:
      if (n == 0 || bl != 0) return ORC_ECORRUPT;
      memset(out, h[1], n);
      break;
    case MODE_RAW:
      if (bl != n || !in_bounds(body, bl, blen)) return ORC_ECORRUPT;
      memcpy(out, blk + body, n);
      break;
    case MODE_RANS: {
      uint32_t maxK = kind == K_LIT ? v->lit_lanes : v->seq_lanes;
      if (K < 1 || K > maxK || n == 0 || !in_bounds(body, bl, blen)) return ORC_ECORRUPT;
      if (K != (uint32_t)orc_rans_lanes(n, maxK, kind == K_LIT ? 16 : 4)) return ORC_ECORRUPT;
      rc = orc_rans_decode(blk + body, bl, n, nw, v->freq[kind], v->P[kind], K, out);
      break;
    }
    default:
      return ORC_ECORRUPT;
  }
  *off = body + ((bl + 15ull) & ~15ull);
  return rc;
}

/* Sequential block decode (plain definition of a block): decode the four
 * streams, then replay the sequences — LL literals, then ML bytes copied
 * byte by byte from absolute position OF: out[p+k] = out[OF+k].  Checks: OF
 * earlier than the write position, ML >= m except a final ML = 0, every
 * earlier block touched by a source listed in the block's dependencies, the
 * block filled exactly, all literals used, and the block's FNV-1a-64. */
static int decode_block(const view_t* v, uint64_t b, uint8_t* out,
                        uint8_t* lit, uint8_t* cmd, uint8_t* mln, uint8_t* ofs) {
  const uint8_t* e = v->a + v->dir + b * DIR_ENTRY;
  uint64_t po = get64(e), pl = get32(e + 8);
  uint32_t ns = get32(e + 12), nl = get32(e + 16);
  const uint64_t B = 1ull << v->bl, sb = b << v->bl;
  const uint64_t eb = sb + B < v->n ? sb + B : v->n;
  if (nl > eb - sb || ns > eb - sb + 1) return ORC_ECORRUPT;
  const uint8_t* blk = v->a + v->payload + po;
  uint64_t off = 0;
  int rc = read_stream(v, K_CMD, blk, pl, &off, 2 * ns, cmd);
  if (!rc) rc = read_stream(v, K_MLEN, blk, pl, &off, 2 * ns, mln);
  if (!rc) rc = read_stream(v, K_OFF, blk, pl, &off, v->w * ns, ofs);
  if (!rc) rc = read_stream(v, K_LIT, blk, pl, &off, nl, lit);
  if (rc) return rc;
  uint64_t d0 = get64(v->a + v->dep_ptr + 8 * b), d1 = get64(v->a + v->dep_ptr + 8 * (b + 1));
  uint64_t p = sb, lc = 0;
  for (uint32_t j = 0; j < ns; j++) {
    uint64_t LL = cmd[j] | (uint64_t)cmd[ns + j] << 8;
    uint64_t ML = mln[j] | (uint64_t)mln[ns + j] << 8;
    uint64_t OF = 0;
    for (uint32_t k = 0; k < v->w; k++) OF |= (uint64_t)ofs[k * ns + j] << (8 * k);
    if (LL > eb - p || lc + LL > nl) return ORC_ECORRUPT;
    memcpy(out + p, lit + lc, LL);
    p += LL;
    lc += LL;
    if (ML == 0) {
      if (j != ns - 1 || OF != 0) return ORC_ECORRUPT;
      continue;
    }
    if (ML < v->m || ML > eb - p || OF >= p) return ORC_ECORRUPT;
    if (OF < sb) {
      uint64_t hi = OF + ML < sb ? OF + ML : sb;
      for (uint64_t a = OF >> v->bl; a <= (hi - 1) >> v->bl; a++) {
        int found = 0;
        for (uint64_t k = d0; k < d1; k++)
          if (get32(v->a + v->dep_idx + 4 * k) == a) { found = 1; break; }
        if (!found) return ORC_ECORRUPT;
      }
    }
    for (uint64_t k = 0; k < ML; k++) out[p + k] = out[OF + k];
    p += ML;
  }
  if (p != eb || lc != nl) return ORC_ECORRUPT;
  if (orc_fnv1a64(out + sb, eb - sb, FNV_BASIS) != get64(e + 24)) return ORC_ECORRUPT;
  return ORC_OK;
}

typedef struct { uint8_t *lit, *cmd, *mln, *ofs; } scratch_t;
static int scratch_alloc(const view_t* v, scratch_t* s) {
  uint64_t B = 1ull << v->bl;
  s->lit = (uint8_t*)malloc(B);
  s->cmd = (uint8_t*)malloc(2 * (B + 1));
  s->mln = (uint8_t*)malloc(2 * (B + 1));
  s->ofs = (uint8_t*)malloc(8 * (B + 1));
  return (s->lit && s->cmd && s->mln && s->ofs) ? 0 : -1;
}
static void scratch_free(scratch_t* s) { free(s->lit); free(s->cmd); free(s->mln); free(s->ofs); }

/* decode_all(A) = x: blocks in file order (a topological order, since every
 * dependency is an earlier block). */
int orc_decode(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap) {
  int rc = orc_validate(a, len);
  if (rc) return rc;
  view_t v;
  open_view(a, len, &v);
  if (cap < v.n) return ORC_ECAPACITY;
  scratch_t s;
  if (scratch_alloc(&v, &s)) { scratch_free(&s); return ORC_EINVAL; }
  for (uint64_t b = 0; b < v.nb && !rc; b++) rc = decode_block(&v, b, out, s.lit, s.cmd, s.mln, s.ofs);
  scratch_free(&s);
  return rc;
}

/* Same bytes, decoded one dependency level at a time with the blocks of a
 * level spread over `threads` OpenMP workers (the CPU form of wavefront
 * decoding). */
int orc_decode_levels(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap, int threads) {
  int rc = orc_validate(a, len);
  if (rc) return rc;
  view_t v;
  open_view(a, len, &v);
  if (cap < v.n) return ORC_ECAPACITY;
  uint64_t* cnt = (uint64_t*)calloc(65, 8);
  uint64_t* order = (uint64_t*)malloc((v.nb ? v.nb : 1) * 8);
  for (uint64_t b = 0; b < v.nb; b++) cnt[get16(a + v.dir + b * DIR_ENTRY + 20) + 1]++;
  for (int L = 0; L < 64; L++) cnt[L + 1] += cnt[L];
  uint64_t* fill = (uint64_t*)calloc(65, 8);
  for (uint64_t b = 0; b < v.nb; b++) {
    uint32_t L = get16(a + v.dir + b * DIR_ENTRY + 20);
    order[cnt[L] + fill[L]++] = b;
  }
  int err = 0;
  for (int L = 0; L < 64; L++) {
    int64_t lo = (int64_t)cnt[L], hi = (int64_t)cnt[L + 1];
    if (lo == hi) continue;
#ifdef _OPENMP
#pragma omp parallel num_threads(threads > 0 ? threads : 1) reduction(| : err)
#endif
    {
      /* every thread of the team reaches the worksharing loop; one whose
       * scratch could not be allocated takes its iterations as failures */
      scratch_t s;
      const int have = scratch_alloc(&v, &s) == 0;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
      for (int64_t i = lo; i < hi; i++)
        if (!have || decode_block(&v, order[i], out, s.lit, s.cmd, s.mln, s.ofs)) err |= 1;
      scratch_free(&s);
    }
  }
  (void)threads;
  free(cnt); free(order); free(fill);
  return err ? ORC_ECORRUPT : ORC_OK;
}

/* Blocks of [lo_blk, hi_blk] plus their dependency closure, marked in mark[]. */
static int mark_closure(const view_t* v, uint8_t* mark, uint64_t lo_blk, uint64_t hi_blk) {
  uint64_t* stack = (uint64_t*)malloc((v->nb ? v->nb : 1) * 8);
  if (!stack) return -1;
  uint64_t sp = 0;
  for (uint64_t b = lo_blk; b <= hi_blk; b++)
    if (!mark[b]) { mark[b] = 1; stack[sp++] = b; }
  while (sp) {
    uint64_t b = stack[--sp];
    uint64_t d0 = get64(v->a + v->dep_ptr + 8 * b), d1 = get64(v->a + v->dep_ptr + 8 * (b + 1));
    for (uint64_t k = d0; k < d1; k++) {
      uint64_t d = get32(v->a + v->dep_idx + 4 * k);
      if (d >= b) { free(stack); return -1; }
      if (!mark[d]) { mark[d] = 1; stack[sp++] = d; }
    }
  }
  free(stack);
  return 0;
}

static int decode_marked(const view_t* v, const uint8_t* mark, uint8_t* scratch, uint64_t* count) {
  scratch_t s;
  if (scratch_alloc(v, &s)) { scratch_free(&s); return ORC_EINVAL; }
  int rc = ORC_OK;
  uint64_t c = 0;
  for (uint64_t b = 0; b < v->nb && !rc; b++)
    if (mark[b]) { rc = decode_block(v, b, scratch, s.lit, s.cmd, s.mln, s.ofs); c++; }
  scratch_free(&s);
  if (count) *count = c;
  return rc;
}

/* Range decode: x[off, off+len), using only the covering blocks and their
 * dependency closure (Position-Invariant Random Access section; the closure
 * is needed because a block's matches may reach into earlier blocks).  The
 * caller validates the archive once (orc_validate) before range calls. */
int orc_decode_range(const uint8_t* a, uint64_t alen, uint64_t off, uint64_t len,
                     uint8_t* scratch, uint8_t* out, uint64_t* closure_blocks) {
  view_t v;
  int rc = open_view(a, alen, &v);
  if (rc) return rc;
  if (off > v.n || len > v.n - off) return ORC_ERANGE;
  if (closure_blocks) *closure_blocks = 0;
  if (len == 0) return ORC_OK;
  uint8_t* mark = (uint8_t*)calloc(v.nb, 1);
  if (!mark) return ORC_EINVAL;
  if (mark_closure(&v, mark, off >> v.bl, (off + len - 1) >> v.bl)) { free(mark); return ORC_EFORMAT; }
  rc = decode_marked(&v, mark, scratch, closure_blocks);
  if (!rc) memcpy(out, scratch + off, len);
  free(mark);
  return rc;
}

/* Read lookup: read r is the 4-line record [idx[r], idx[r+1]).  Output is
 * the records in request order; offsets[j] = bytes before record j. */
int orc_read_lookup(const uint8_t* a, uint64_t alen, const int64_t* ids, uint64_t n,
                    uint8_t* scratch, uint8_t* out, uint64_t cap, uint64_t* offsets) {
  view_t v;
  int rc = open_view(a, alen, &v);
  if (rc) return rc;
  if (v.kind != 1) return ORC_ENOINDEX;
  offsets[0] = 0;
  for (uint64_t j = 0; j < n; j++) {
    if (ids[j] < 0 || (uint64_t)ids[j] >= v.n_reads) return ORC_ERANGE;
    uint64_t r = (uint64_t)ids[j];
    offsets[j + 1] = offsets[j] + get64(a + v.ridx + 8 * (r + 1)) - get64(a + v.ridx + 8 * r);
  }
  if (offsets[n] > cap) return ORC_ECAPACITY;
  if (n == 0) return ORC_OK;
  uint8_t* mark = (uint8_t*)calloc(v.nb ? v.nb : 1, 1);
  if (!mark) return ORC_EINVAL;
  for (uint64_t j = 0; j < n && !rc; j++) {
    uint64_t r = (uint64_t)ids[j];
    uint64_t s = get64(a + v.ridx + 8 * r), e = get64(a + v.ridx + 8 * (r + 1));
    if (mark_closure(&v, mark, s >> v.bl, (e - 1) >> v.bl)) rc = ORC_EFORMAT;
  }
  if (!rc) rc = decode_marked(&v, mark, scratch, NULL);
  for (uint64_t j = 0; j < n && !rc; j++) {
    uint64_t r = (uint64_t)ids[j];
    uint64_t s = get64(a + v.ridx + 8 * r);
    memcpy(out + offsets[j], scratch + s, offsets[j + 1] - offsets[j]);
  }
  free(mark);
  return rc;
}
