/*
 * liblz — device-resident decoder for the absolute-offset block LZ77 codec
 * (arXiv 2606.18900), on one AMD Instinct MI355X (gfx950).
 *
 * The method (paper, Background section): every LZ77 back-reference is an
 * absolute position in the decompressed output; the output is cut into
 * fixed-size blocks (Block Granularity section: 16 KB); each block stores four
 * streams (literals, match lengths, absolute offsets, command sequence); a
 * block can be decoded once the blocks holding its source bytes are done.
 * This library decodes entirely on the GPU (Full Device-Resident Pipeline
 * section): entropy decode and match resolution, ordered by dependency level
 * ("wavefronts"), plus block-range decode and read-level random access through
 * a read -> record-start index (Position-Invariant Random Access section and
 * its Read-Level Index subsection), and range decode into a capped output
 * window (Scale section).
 *
 * Conventions
 *  - Every function returns an int status: LZ_OK (0) or a negative LZ_E* code;
 *    lz_last_error() gives the text of the last failure of the calling thread.
 *  - The caller owns every device buffer (archive, workspace, outputs,
 *    scratch); the library never allocates device memory.  The one device
 *    buffer it holds is the fixed scratch array of lz_read_lookup_noalloc,
 *    part of its code object.  A handle keeps non-owning pointers to the
 *    archive and workspace, which must outlive it.
 *  - Device calls are asynchronous on the caller's HIP stream `s` (may be 0).
 *    Arguments are checked on the host before anything is enqueued; errors
 *    found by a kernel (corrupt payload, scratch exhausted, watchdog) are
 *    latched in the workspace status word and returned by lz_sync_status().
 *  - Offsets and sizes are bytes, 64-bit (Scale section: 64-bit fields).
 *  - Calls on one handle must not overlap in time (one stream, or ordered
 *    streams); different handles are independent.
 */
#ifndef LZ_H
#define LZ_H
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LZ_OK        0
#define LZ_EINVAL   (-1)  /* bad argument, null pointer, misaligned buffer   */
#define LZ_EFORMAT  (-2)  /* bad magic/version/checksum or broken invariant   */
#define LZ_ECAPACITY (-3) /* output/workspace/scratch too small; see *needed  */
#define LZ_ERANGE   (-4)  /* offset+len > N, or read id outside [0, n_reads)  */
#define LZ_ENOINDEX (-5)  /* archive has no read index (not FASTQ)            */
#define LZ_EDEVICE  (-6)  /* HIP runtime error; text in lz_last_error()       */
#define LZ_ECORRUPT (-7)  /* device-side decode check failed                  */
#define LZ_EBUDGET  (-8)  /* serving admission refused (budget)               */

/* Encoder parameters (container format v2).  The match search is global and
 * greedy with absolute source positions (Background section); blocks are
 * 2^block_log2 bytes (16 KB in the paper); levels are capped at max_level-1. */
typedef struct lz_params {
  uint32_t block_log2;    /* 6..15; the device decoder takes 6..14           */
  uint32_t max_level;     /* D, 1..64                                        */
  uint32_t min_match;     /* m, hash_len..255                                */
  uint32_t hash_len;      /* 4..16                                           */
  uint32_t hash_bits;     /* 8..30                                           */
  uint32_t chain_depth;   /* 0 = unbounded                                   */
  uint32_t window_log2;   /* 0 = unbounded                                   */
  uint32_t lit_lanes;     /* max rANS lanes, literal stream, 1..256          */
  uint32_t seq_lanes;     /* max rANS lanes, CMD/MLEN/OFF, 1..64             */
  uint32_t prob_bits[4];  /* LIT, CMD, MLEN, OFF; 8..12                      */
  uint32_t kind;          /* 0 raw, 1 FASTQ (writes the read index), 2 FASTA */
  uint32_t level_penalty; /* beta: match score = length - beta * level       */
  uint32_t threads;       /* encoder host threads (0 = all); no effect on bytes */
  uint32_t segment_log2;  /* 0: the global parse defined above (bytes equal to
                             the reference policy, memory ~20 B per input byte);
                             block_log2..24: segmented parse with bounded
                             memory (see lz_encode), for inputs of many GB    */
} lz_params;

typedef struct lz_info {
  uint64_t n;               /* decompressed bytes N                          */
  uint64_t n_blocks;        /* ceil(N / B)                                   */
  uint64_t n_reads;         /* FASTQ records (0 without a read index)        */
  uint64_t archive_len;     /* total archive bytes                           */
  uint64_t source_fnv;      /* FNV-1a-64 over the LE64 block hashes          */
  uint64_t workspace_bytes; /* device workspace lz_open needs                */
  uint64_t literal_bytes;   /* sum of literal-stream lengths (lz_get_info only);
                               N - literal_bytes = bytes copied by matches    */
  uint64_t payload_bytes;   /* compressed block payload bytes                 */
  uint32_t block_log2, max_level, n_levels, offset_width, max_record_len, kind;
} lz_info;

/* One request of a batch: kind 0 = read lookup (a = read id), kind 1 = byte
 * range (a = offset, b = length).  Results are concatenated in request order. */
typedef struct lz_request {
  int64_t kind, a, b;
} lz_request;

/* Launch knobs (chosen by the autotuner; none of them changes a decoded byte). */
typedef struct lz_tuning {
  uint32_t sync_mode;   /* whole-file decode: 0 = one launch per dependency
                           level (lz_open's default), 1 = one cooperative
                           launch with a grid barrier between levels      */
  uint32_t wg_per_cu;   /* grid = wg_per_cu * CUs workgroups (a level launch
                           takes at most its block count); 1..4, default 3   */
  uint32_t spin_limit;  /* watchdog: max polls of a dependency flag before the
                           kernel gives up with LZ_ECORRUPT (0 = default)     */
  uint32_t req_sync_mode; /* request calls (ranges, reads, batches): the same
                           two modes for the closure decode; default 0     */
  uint32_t plan_blocks; /* request calls expected to cover at most this many
                           blocks are planned by one workgroup in one launch,
                           larger ones by the eight-kernel path; 1..2^20, 0 =
                           default 4096                                     */
} lz_tuning;

typedef struct lz_handle lz_handle;

/* ---- host ------------------------------------------------------------- */

/* Fill *p with the default profile: 16 KB blocks, D = 64, m = h = 16,
 * hash_bits 20, chain 64, no window, 256/64 lanes, P = 12/10/10/10,
 * level_penalty 32. */
int lz_params_default(lz_params* p);

/* Compress src[0..n) (host memory).  On success *archive (host memory owned by
 * the library, free with lz_free) holds *archive_len bytes.  Errors: EINVAL
 * (bad parameters, or kind FASTQ and the input is not whole 4-line records).
 * With segment_log2 > 0 the input is parsed in segments of 2^segment_log2
 * bytes on host threads: a match source is an earlier position of the same
 * segment (hash chain, most recent first) or the first position ever seen with
 * the same hash, if that lies 32 or more segments back; the scoring and level
 * rules are those of the global parse.  The output does not depend on the
 * thread count; working memory is bounded by the segment size, the hash table
 * (8 B x 2^hash_bits) and the archive itself. */
int lz_encode(const uint8_t* src, uint64_t n, const lz_params* p,
              uint8_t** archive, uint64_t* archive_len);
void lz_free(void* p);

/* Parse the 128-byte header of a host copy of an archive (len >= 128) and
 * report sizes, including the workspace lz_open needs.  EFORMAT on a bad header. */
int lz_info_get(const uint8_t* host_archive, uint64_t len, lz_info* out);

/* ---- device ----------------------------------------------------------- */

/* Bind an archive already in device memory.  Copies header, directory and
 * dependency lists to the host once and validates every container invariant
 * (EFORMAT), checks device limits (EFORMAT: block_log2 > 14, N >= 2^40, more
 * than 1025 sequences per block possible), then builds the level-ordered block queue and the rANS
 * lookup tables in the workspace (d_ws, ws_len bytes, 256-byte aligned;
 * ECAPACITY if smaller than lz_info.workspace_bytes).  Synchronises s. */
int lz_open(const uint8_t* d_archive, uint64_t len, void* d_ws, uint64_t ws_len,
            hipStream_t s, lz_handle** h);
int lz_close(lz_handle* h);
int lz_get_info(const lz_handle* h, lz_info* out);
int lz_set_tuning(lz_handle* h, const lz_tuning* t);
int lz_get_tuning(const lz_handle* h, lz_tuning* t);

/* Whole-file decode (Mode 2 of the Full Device-Resident Pipeline section):
 * d_out[0..N) = x.  d_out must be 16-byte aligned, cap >= N (else ECAPACITY). */
int lz_decode_all(lz_handle* h, uint8_t* d_out, uint64_t cap, hipStream_t s);

/* Range decode (Position-Invariant Random Access section): d_out[0..len) =
 * x[offset, offset+len).  Decodes the covering blocks plus their dependency
 * closure; blocks that cannot go straight into d_out are decoded into
 * d_scratch (16-byte aligned, scratch_len bytes; one block-sized slot per such
 * block).  len = 0 is a no-op.  ERANGE if offset + len > N.  A scratch shortage
 * found on the device is reported by lz_sync_status as ECAPACITY. */
int lz_decode_range(lz_handle* h, uint64_t offset, uint64_t len, uint8_t* d_out,
                    void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* Read lookup (Read-Level Index subsection): for d_ids[0..n) (device, int64)
 * write the 4-line records, concatenated in request order, to d_out and their
 * exclusive prefix offsets to d_offsets[0..n] (device, u64).  cap must be >=
 * n * max_record_len (ECAPACITY otherwise).  ENOINDEX without a read index;
 * an id outside [0, n_reads) is latched as ERANGE on the device. */
int lz_read_lookup(lz_handle* h, const int64_t* d_ids, uint64_t n, uint8_t* d_out,
                   uint64_t cap, uint64_t* d_offsets, void* d_scratch,
                   uint64_t scratch_len, hipStream_t s);

/* Allocation-free read lookup, for callers that cannot allocate device memory
 * per call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result as lz_read_lookup, but the request scratch
 * is a fixed array of LZ_NOALLOC_SCRATCH_BYTES that the library holds in
 * device memory, one per GPU, for the life of the process.  n is at most
 * LZ_NOALLOC_MAX_IDS (ECAPACITY otherwise); a dependency closure needing more
 * block slots than the array holds after the per-request tables (2039 slots of
 * 16 KiB) is latched as ECAPACITY.  The current device must be the one the
 * handle was opened on.  Every call on a GPU shares that GPU's array: calls
 * that overlap in time on one GPU (any handle, any stream) race and must be
 * ordered by the caller.  No device or host allocation is made by the call. */
#define LZ_NOALLOC_SCRATCH_BYTES (32u << 20)
#define LZ_NOALLOC_MAX_IDS 4096
int lz_read_lookup_noalloc(lz_handle* h, const int64_t* d_ids, uint64_t n, uint8_t* d_out,
                           uint64_t cap, uint64_t* d_offsets, hipStream_t s);

/* ---- FASTA coordinate access (chr:pos) ----------------------------------
 * The paper leaves coordinate-based access to FASTA as future work (Read-Level
 * Index subsection).  A sequence of a FASTA file is described as in a .fai
 * index: byte offset of its first base, number of bases, bases per full line
 * and bytes per full line (bases + newline).  Base k of the sequence then lies
 * at byte offset + (k / line_bases) * line_bytes + k % line_bases. */
typedef struct lz_fasta_seq {
  char name[64];          /* NUL-terminated, truncated to 63 bytes            */
  uint64_t offset;        /* byte offset of the first base                     */
  uint64_t length;        /* bases                                            */
  uint32_t line_bases;    /* bases per full line (0 if the lines are uneven)  */
  uint32_t line_bytes;    /* bytes per full line                              */
} lz_fasta_seq;

/* Host: scan a FASTA text (records '>' name line, then sequence lines ending
 * in '\n') and describe its sequences; writes min(count, cap) entries, *count
 * receives the total.  EINVAL if the text does not start with '>'. */
int lz_fasta_index(const uint8_t* src, uint64_t n, lz_fasta_seq* out, uint64_t cap,
                   uint64_t* count);

/* Device: d_out[0 .. end-start) = bases [start, end) of sequence *sq (no
 * newlines): the covering byte range is decoded with lz_decode_range into the
 * front of d_scratch, then the bases are gathered by line arithmetic.
 * ERANGE if end > sq->length or start > end; ENOINDEX if the sequence's lines
 * are uneven (line_bases 0).  d_scratch needs the covering byte range rounded
 * up to 256 bytes plus the scratch of a range decode. */
int lz_decode_region(lz_handle* h, const lz_fasta_seq* sq, uint64_t start, uint64_t end,
                     uint8_t* d_out, void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* Batched requests (mixed reads and ranges) resolved together: one closure
 * over all requests, one decode launch over the shared level-ordered queue,
 * then a gather into d_out at d_offsets (device, n+1 entries).  d_reqs is a
 * device array of n lz_request.  n_max sizes the device-side request
 * capacity the call was planned for (n <= n_max); the sequence of launches
 * depends only on (handle, n_max), so it can be captured once in a HIP graph
 * and replayed with new request contents.  cap bounds the output; a larger
 * total is latched as ECAPACITY. */
int lz_decode_batch(lz_handle* h, const lz_request* d_reqs, const uint32_t* d_n,
                    uint64_t n_max, uint8_t* d_out, uint64_t cap, uint64_t* d_offsets,
                    void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* Per-block FNV-1a-64 of d_out[0..N) compared on the device with the
 * directory's source hashes (Experimental Setup: FNV on device paths);
 * mismatches are latched as ECORRUPT.  *d_tree (device u64) receives the
 * tree hash.  d_scratch needs 8 * n_blocks bytes. */
int lz_verify(lz_handle* h, const uint8_t* d_out, uint64_t* d_tree,
              void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* The same check for a decoded part of the file: d_out holds x[offset,
 * offset+len), offset a multiple of the block size and len one too unless the
 * range ends at N (EINVAL otherwise); every block of the range is hashed and
 * compared with its source hash (mismatch latched as ECORRUPT).  d_scratch
 * needs 8 bytes per block of the range. */
int lz_verify_range(lz_handle* h, const uint8_t* d_out, uint64_t offset, uint64_t len,
                    void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* Work of the last request call on h (lz_decode_range, lz_read_lookup,
 * lz_read_lookup_noalloc, lz_decode_batch): closure_blocks = blocks decoded
 * (the covering blocks plus their dependency closure, Position-Invariant
 * Random Access section), scratch_slots = those decoded into scratch, covering
 * = (request, covering block) pairs.  Synchronises s. */
typedef struct lz_stats {
  uint64_t closure_blocks, scratch_slots, covering;
} lz_stats;
int lz_last_stats(lz_handle* h, lz_stats* out, hipStream_t s);

/* Synchronise s, return and clear the latched device status (LZ_OK if none). */
int lz_sync_status(lz_handle* h, hipStream_t s);

const char* lz_last_error(void);

/* ---- stream-separated FASTQ (Discussion, "Where ACEAPEX Stands on Ratio":
 * read ids, sequences and quality strings stored apart gain ratio with the
 * same codec) ------------------------------------------------------------
 *
 * A split container holds a 4-line FASTQ file as four kind-0 archives of its
 * line streams -- H (id lines), S (sequence lines), P ('+' lines), Q (quality
 * lines), each line with its newline -- plus a read index of two u64 tables:
 * hstart[i], sstart[i] = offsets of record i's id and sequence lines in H
 * and S (n_reads + 1 entries each).  Record i's P and Q lines start at 2 i
 * and sstart[i]; its first file byte is hstart[i] + 2 sstart[i] + 2 i.
 * Layout (little-endian): "LZSF", u16 version 2, u16 flags 3, u64 N, u64
 * n_reads, u64 offsets of hstart[] and sstart[], u64 archive offsets[4]
 * (multiples of 256) and lengths[4], u64 FNV-1a-64 of the source, u32
 * longest record, u32 0, u64 FNV-1a-64 of bytes 0..119; then the tables and
 * the archives, gaps zero. */
typedef struct lz_split lz_split;

typedef struct lz_split_info {
  uint64_t n;                /* file bytes N                                   */
  uint64_t n_reads;          /* records                                        */
  uint64_t container_len;    /* total container bytes                          */
  uint64_t source_fnv;       /* FNV-1a-64 of the whole file                    */
  uint64_t workspace_bytes;  /* device workspace lz_split_open needs (the four
                                decoded streams, then four lz_open workspaces) */
  uint64_t stream_len[4];    /* decoded bytes of H, S, P, Q                    */
  uint64_t archive_len[4];   /* their archive bytes                            */
  uint32_t max_record_len;   /* longest record (file bytes)                    */
  uint32_t reserved;
} lz_split_info;

/* Host: write the split container of a FASTQ text (records of 4 lines, each
 * ending in '\n').  Every stream is encoded by lz_encode with *p and kind 0.
 * EINVAL for text that is not whole records, an id line without '@', a
 * third line other than a bare '+', or a quality line whose length differs
 * from its sequence line's.  *out is malloc'd (free with lz_free). */
int lz_encode_split(const uint8_t* src, uint64_t n, const lz_params* p, uint8_t** out,
                    uint64_t* out_len);

/* Device: read and check the container's headers from d_container (device,
 * len bytes; synchronises s) and describe it. */
int lz_split_info_get(const uint8_t* d_container, uint64_t len, hipStream_t s, lz_split_info* out);

/* Bind a device-resident container (256-byte aligned) and a caller workspace
 * of lz_split_info.workspace_bytes (256-byte aligned): the record tables are
 * copied to the host and checked against the streams, each stream archive is
 * opened with lz_open.  Synchronises s. */
int lz_split_open(const uint8_t* d_container, uint64_t len, void* d_ws, uint64_t ws_len, hipStream_t s,
                  lz_split** out);
int lz_split_close(lz_split* sp);

/* The lz_handle of stream k (0 H, 1 S, 2 P, 3 Q), owned by sp: for tuning
 * and statistics. */
int lz_split_stream(lz_split* sp, uint32_t k, lz_handle** out);

/* d_out[0..N) = the FASTQ file: the four streams are decoded into the
 * workspace (lz_decode_all each), then the records are reassembled in file
 * order on the device. */
int lz_split_decode_all(lz_split* sp, uint8_t* d_out, uint64_t cap, hipStream_t s);

/* Scratch (bytes, 256-byte aligned buffer) of lz_split_decode_range (n = 1)
 * and of lz_split_read_lookup for n ids. */
int lz_split_scratch_bytes(const lz_split* sp, uint64_t n, uint64_t* bytes);

/* d_out[0..len) = file bytes [offset, offset + len): the records covering the
 * range are found in the host copy of the read index, their lines decoded
 * from each stream with lz_decode_range (dependency closure included) and
 * reassembled.  ERANGE if the range leaves the file. */
int lz_split_decode_range(lz_split* sp, uint64_t offset, uint64_t len, uint8_t* d_out, void* d_scratch,
                          uint64_t scratch_len, hipStream_t s);

/* Records d_ids[0..n) (device int64): every stream answers a batch of range
 * requests (lz_decode_batch) for the ids' lines, then record k is assembled
 * at d_out[d_offsets[k] .. d_offsets[k+1]) (d_offsets: device, n + 1 u64).
 * cap >= n * max_record_len.  An id outside [0, n_reads) is latched as
 * ERANGE (lz_split_sync_status) and yields an empty record. */
int lz_split_read_lookup(lz_split* sp, const int64_t* d_ids, uint64_t n, uint8_t* d_out, uint64_t cap,
                         uint64_t* d_offsets, void* d_scratch, uint64_t scratch_len, hipStream_t s);

/* lz_sync_status of the four streams: the first failure, all cleared. */
int lz_split_sync_status(lz_split* sp, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif
