/*
 * Plain CPU oracle for the absolute-offset block LZ77 codec.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its
 * Python binding, the benchmark's timed path) may include, link, load or call
 * this code; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no source with the product.
 *
 * What it computes (paper: Background section; 64-bit fields: Scale section):
 *   - an encoder doing a global hash-chain match search whose matches carry the
 *     absolute source position in the decompressed output, cut into fixed-size
 *     blocks, each block stored as four entropy-coded streams (literals, match
 *     lengths, absolute offsets, command sequence = literal-run lengths);
 *   - a sequential decoder: decode_all(A) == x by definition;
 *   - a validator for every container invariant;
 *   - the read -> record-start index (Read-Level Index section: 8 bytes/read);
 *   - FNV-1a-64 block hashes (Experimental Setup: FNV on device paths).
 * Every step the paper leaves open follows the readings listed in the design
 * notes (container format v2); each function below names its step.
 */
#ifndef LZ_ORACLE_H
#define LZ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_EINVAL = -1, ORC_EFORMAT = -2, ORC_ECAPACITY = -3,
  ORC_ERANGE = -4, ORC_ENOINDEX = -5, ORC_ECORRUPT = -7
};

typedef struct orc_params {
  uint32_t block_log2;   /* B = 2^block_log2, 6..15                        */
  uint32_t max_level;    /* D: levels are 0..D-1, 1..64                    */
  uint32_t min_match;    /* m >= hash_len                                  */
  uint32_t hash_len;     /* h, 4..16                                       */
  uint32_t hash_bits;    /* H, 8..30                                       */
  uint32_t chain_depth;  /* C, 0 = unbounded                               */
  uint32_t window_log2;  /* R, 0 = unbounded                               */
  uint32_t lit_lanes;    /* max rANS lanes of the literal stream, 1..256   */
  uint32_t seq_lanes;    /* max rANS lanes of CMD/MLEN/OFF, 1..64          */
  uint32_t prob_bits[4]; /* P for LIT, CMD, MLEN, OFF; 8..12               */
  uint32_t kind;         /* 0 raw, 1 FASTQ (builds the read index), 2 FASTA */
  uint32_t level_penalty;/* beta: candidate score = length - beta * level   */
} orc_params;

typedef struct orc_info {
  uint64_t n, n_blocks, n_reads, total_len, source_fnv;
  uint32_t block_log2, max_level, n_levels, offset_width, max_record_len, kind;
} orc_info;

void     orc_params_default(orc_params* p);
uint64_t orc_fnv1a64(const uint8_t* p, uint64_t n, uint64_t h);
uint64_t orc_fnv_basis(void);

/* Entropy stage pieces, exposed for the unit pins. */
int orc_normalize(const uint64_t* counts, uint32_t prob_bits, uint16_t* freq);
int orc_rans_lanes(uint32_t n, uint32_t max_lanes, uint32_t per_lane);
int orc_rans_encode(const uint8_t* sym, uint32_t n, const uint16_t* freq,
                    uint32_t prob_bits, uint32_t lanes, uint8_t** body,
                    uint64_t* body_len, uint32_t* n_words);
int orc_rans_decode(const uint8_t* body, uint64_t body_len, uint32_t n,
                    uint32_t n_words, const uint16_t* freq, uint32_t prob_bits,
                    uint32_t lanes, uint8_t* out);

/* Parse only: the greedy hash-chain parse with the level cap.  Returns arrays
 * (owned by the caller, free with orc_free) of n_seq entries: block id, LL, ML, OF. */
/* Source rebasing of a parse (see oracle.c), in place on `of`. */
void orc_rebase(uint64_t n_seq, const uint32_t* blk, const uint32_t* ll, const uint32_t* ml,
                uint64_t* of, uint32_t block_log2);
int orc_parse(const uint8_t* src, uint64_t n, const orc_params* p,
              uint64_t* n_seq, uint32_t** blk, uint32_t** ll, uint32_t** ml,
              uint64_t** of, uint16_t** level);

int  orc_encode(const uint8_t* src, uint64_t n, const orc_params* p,
                uint8_t** archive, uint64_t* archive_len);
int  orc_validate(const uint8_t* a, uint64_t len);
int  orc_info_get(const uint8_t* a, uint64_t len, orc_info* out);
int  orc_decode(const uint8_t* a, uint64_t len, uint8_t* out, uint64_t cap);
/* Decode levels in turn with `threads` OpenMP workers per level (timing only;
 * the bytes are those of orc_decode). */
int  orc_decode_levels(const uint8_t* a, uint64_t len, uint8_t* out,
                       uint64_t cap, int threads);
/* x[off, off+len): decodes the covering blocks and their dependency closure
 * into `scratch` (N bytes, caller-owned) and copies the range out. */
int  orc_decode_range(const uint8_t* a, uint64_t alen, uint64_t off,
                      uint64_t len, uint8_t* scratch, uint8_t* out,
                      uint64_t* closure_blocks);
/* Records ids[0..n) concatenated; offsets[n+1] exclusive prefix sums. */
int  orc_read_lookup(const uint8_t* a, uint64_t alen, const int64_t* ids,
                     uint64_t n, uint8_t* scratch, uint8_t* out, uint64_t cap,
                     uint64_t* offsets);
void orc_free(void* p);

#ifdef __cplusplus
}
#endif
#endif
